/*
 * Complex-step derivatives of the second-order hybrid step (Eq. 7) of
 * Grimm & Stadel, "The GENGA Code" (arXiv:1404.2324): the oracle of the
 * encounter-aware adjoint.  The paper has no adjoint; what is defined here
 * is the derivative of the step of genga_oracle.c (go_massive_step) with
 * respect to the initial democratic state and the masses, with every
 * discrete decision of the step held where it falls.
 *
 * TEST INFRASTRUCTURE ONLY, like genga_oracle.c, and sharing no code with
 * the GPU library.
 *
 * Method: for a real map f, f(z + i h d) = f(z) + i h J d + O(h^2), so
 * J d = Im f(z + i h d) / h with no subtraction and no truncation error for
 * a tiny h (the complex-step derivative: Squire and Trapp, SIAM Review 40,
 * 1998).  The step of genga_oracle.c is written again below in complex
 * arithmetic.  Sums, products and quotients of complex numbers whose
 * imaginary parts are ~h smaller than their real parts have real parts equal
 * to the real operation's result (the h^2 cross terms are far below half an
 * ulp), so with -ffp-contract=off the real part of every quantity is the
 * real oracle's value bit for bit.  The functions that are not rational
 * (square and cube roots) are continued to first order by hand from their
 * real values, which keeps that property.  Every decision is taken on real
 * parts: the branches of the changeover function, the larger of two radii
 * and of the two terms of Eq. (6), the candidate and encounter tests
 * (Eqs. 10-12), the groups (App. A), the acceptance and halving of BS
 * attempts, and the stopping of the Kepler iteration.  The Kepler equation
 * is solved in real arithmetic; the imaginary part of its root follows from
 * the implicit function theorem, -Im F / F' at the real root.
 *
 * Pinned by (tests/test_oracle_pins.py): real parts equal to go_massive_step
 * bit for bit; with K == 1 the directional derivative equals the tangent-
 * linear model go_free_tlm; with encounters and BS groups it agrees with
 * central differences of go_massive_step.
 */
#include "genga_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define C3(a, i) (&(a)[3 * (size_t)(i)])

/* first-order continuations of the roots: f(a + ib) = f(a) + i b f'(a) */
static cplx c_sqrt(cplx z) {
    double a = creal(z), s = sqrt(a);
    return CMPLX(s, cimag(z) / (2.0 * s));
}
static cplx c_cbrt(cplx z) {
    double a = creal(z), c = cbrt(a);
    return CMPLX(c, cimag(z) / (3.0 * c * c));
}
static cplx c_dot3(const cplx *a, const cplx *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Eq. (4) with y of Eq. (5), as go_changeover / pair_K */
static void c_changeover(cplx y, cplx *K, cplx *dKdy) {
    if (creal(y) <= 0.0) {
        *K = 0.0;
        *dKdy = 0.0;
    } else if (creal(y) >= 1.0) {
        *K = 1.0;
        *dKdy = 0.0;
    } else {
        cplx D = 2.0 * y * y - 2.0 * y + 1.0;
        *K = y * y / D;
        *dKdy = 2.0 * y * (1.0 - y) / (D * D);
    }
}

static void c_pair_K(cplx r, cplx rcij, cplx *K, cplx *dKdr) {
    if (!(creal(rcij) > 0.0)) {
        *K = 1.0;
        *dKdr = 0.0;
        return;
    }
    cplx y = (r - 0.1 * rcij) / (0.9 * rcij);
    cplx dKdy;
    c_changeover(y, K, &dKdy);
    *dKdr = dKdy / (0.9 * rcij);
}

static cplx c_max(cplx a, cplx b) { return creal(a) > creal(b) ? a : b; }

/* Eq. (6), as go_rcrit */
static void c_rcrit(const go_params *p, int n, const cplx *m, const cplx *x, const cplx *v,
                    cplx *rc) {
    double mu = p->G * p->m0;
    for (int i = 0; i < n; ++i) {
        cplx r = c_sqrt(c_dot3(C3(x, i), C3(x, i)));
        cplx vv = c_dot3(C3(v, i), C3(v, i));
        cplx inva = 2.0 / r - vv / mu;
        cplx a = creal(inva) > 0.0 ? 1.0 / inva : r;
        cplx rh = a * c_cbrt(m[i] / (3.0 * p->m0));
        cplx rv = p->n2 * fabs(p->dt) * c_sqrt(vv);
        cplx r1 = p->n1 * rh;
        rc[i] = creal(r1) > creal(rv) ? r1 : rv;
    }
}

/* H_B acceleration (gradient of Eq. 2), as go_accel */
static void c_accel(const go_params *p, int n, const cplx *m, const cplx *x, const cplx *rc,
                    cplx *acc) {
    for (int i = 0; i < n; ++i) {
        cplx a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            cplx d0 = x[3 * j + 0] - x[3 * i + 0];
            cplx d1 = x[3 * j + 1] - x[3 * i + 1];
            cplx d2 = x[3 * j + 2] - x[3 * i + 2];
            cplx r2 = d0 * d0 + d1 * d1 + d2 * d2;
            cplx r = c_sqrt(r2);
            cplx f;
            if (p->encounter_free) {
                f = 1.0 / (r2 * r);
            } else {
                cplx rcij = c_max(rc[i], rc[j]);
                cplx K, dK;
                c_pair_K(r, rcij, &K, &dK);
                f = K / (r2 * r) - dK / r2;
            }
            cplx s = p->G * m[j] * f;
            a0 += s * d0;
            a1 += s * d1;
            a2 += s * d2;
        }
        acc[3 * i + 0] = a0;
        acc[3 * i + 1] = a1;
        acc[3 * i + 2] = a2;
    }
}

/* H_C flow (Eq. 3), as go_sun_drift */
static void c_sun_drift(const go_params *p, int n, const cplx *m, cplx *x, const cplx *v,
                        double h) {
    cplx P[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < 3; ++k) P[k] += m[j] * v[3 * j + k];
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) x[3 * i + k] += h * P[k] / p->m0;
}

/* Stumpff functions, as go_stumpff (the quartering count from |Re z|) */
static void c_stumpff(cplx z, cplx c[4]) {
    int nq = 0;
    while (fabs(creal(z)) >= 0.1 && nq < 64) {
        z *= 0.25;
        ++nq;
    }
    cplx c2 = 0.0, c3 = 0.0;
    {
        cplx t2 = 1.0 / 2.0, t3 = 1.0 / 6.0;
        for (int k = 0; k <= 8; ++k) {
            c2 += t2;
            c3 += t3;
            t2 *= -z / ((double)(2 * k + 3) * (double)(2 * k + 4));
            t3 *= -z / ((double)(2 * k + 4) * (double)(2 * k + 5));
        }
    }
    cplx c0 = 1.0 - z * c2;
    cplx c1 = 1.0 - z * c3;
    for (int q = 0; q < nq; ++q) {
        cplx n0 = 2.0 * c0 * c0 - 1.0;
        cplx n1 = c0 * c1;
        cplx n2 = 0.5 * c1 * c1;
        cplx n3 = 0.25 * (c2 + c0 * c3);
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

static void c_gk_at(cplx s, cplx beta, cplx G[4]) {
    cplx c[4];
    c_stumpff(beta * s * s, c);
    G[0] = c[0];
    G[1] = s * c[1];
    G[2] = s * s * c[2];
    G[3] = s * s * s * c[3];
}

/* Kepler drift (Eq. 9 in universal variables), as go_kepler: the root s of
 * the universal Kepler equation is found by go_kepler's own iteration on the
 * real parts; its imaginary part is -Im F(s) / F'(s) at that root. */
static int c_kepler(double mu, const cplx *x0, const cplx *v0, double dt, cplx *x, cplx *v,
                    int max_iter, int *iters) {
    double xr[3], vr[3], s;
    for (int k = 0; k < 3; ++k) {
        xr[k] = creal(x0[k]);
        vr[k] = creal(v0[k]);
    }
    int rcode = go_kepler_root(mu, xr, vr, dt, max_iter, &s, iters);
    cplx r0 = c_sqrt(c_dot3(x0, x0));
    cplx eta0 = c_dot3(x0, v0);
    cplx beta = 2.0 * mu / r0 - c_dot3(v0, v0);
    cplx zeta0 = mu - beta * r0;
    cplx G[4];
    c_gk_at(s, beta, G);
    cplx F = r0 * G[1] + eta0 * G[2] + mu * G[3] - dt;
    cplx Fp = r0 + eta0 * G[1] + zeta0 * G[2];
    cplx sc = CMPLX(s, -cimag(F) / creal(Fp));
    c_gk_at(sc, beta, G);
    cplx r = r0 + eta0 * G[1] + zeta0 * G[2];
    cplx f = 1.0 - mu * G[2] / r0;
    cplx g = dt - mu * G[3];
    cplx fd = -mu * G[1] / (r * r0);
    cplx gd = 1.0 - mu * G[2] / r;
    cplx xn[3], vn[3];
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

/* ---- BS of H_A for one group (Sec. 2.2, 3.2.6), as genga_oracle.c ------ */
#define CS_KMAX 8

typedef struct {
    const go_params *p;
    int ng;
    const cplx *m;
    const cplx *rc;
} c_ha_sys;

static void c_ha_deriv(const c_ha_sys *s, const cplx *y, cplx *dy) {
    int ng = s->ng;
    double Gm0 = s->p->G * s->p->m0;
    for (int i = 0; i < ng; ++i) {
        const cplx *xi = &y[6 * i];
        cplx r2 = c_dot3(xi, xi);
        cplx r = c_sqrt(r2);
        cplx fs = -Gm0 / (r2 * r);
        cplx a0 = fs * xi[0], a1 = fs * xi[1], a2 = fs * xi[2];
        for (int j = 0; j < ng; ++j) {
            if (j == i) continue;
            const cplx *xj = &y[6 * j];
            cplx d0 = xj[0] - xi[0], d1 = xj[1] - xi[1], d2 = xj[2] - xi[2];
            cplx q2 = d0 * d0 + d1 * d1 + d2 * d2;
            cplx q = c_sqrt(q2);
            cplx rcij = c_max(s->rc[i], s->rc[j]);
            cplx K, dK;
            c_pair_K(q, rcij, &K, &dK);
            cplx f = (1.0 - K) / (q2 * q) + dK / q2;
            cplx sj = s->p->G * s->m[j] * f;
            a0 += sj * d0;
            a1 += sj * d1;
            a2 += sj * d2;
        }
        dy[6 * i + 0] = y[6 * i + 3];
        dy[6 * i + 1] = y[6 * i + 4];
        dy[6 * i + 2] = y[6 * i + 5];
        dy[6 * i + 3] = a0;
        dy[6 * i + 4] = a1;
        dy[6 * i + 5] = a2;
    }
}

static void c_mmid(const c_ha_sys *s, const cplx *y0, double H, int nsub, cplx *yout, cplx *ym,
                   cplx *yn, cplx *d, cplx *tmp) {
    int dim = 6 * s->ng;
    double hs = H / nsub;
    c_ha_deriv(s, y0, d);
    for (int k = 0; k < dim; ++k) {
        ym[k] = y0[k];
        yn[k] = y0[k] + hs * d[k];
    }
    for (int m = 1; m < nsub; ++m) {
        c_ha_deriv(s, yn, d);
        for (int k = 0; k < dim; ++k) {
            tmp[k] = ym[k] + 2.0 * hs * d[k];
            ym[k] = yn[k];
            yn[k] = tmp[k];
        }
    }
    c_ha_deriv(s, yn, d);
    for (int k = 0; k < dim; ++k) yout[k] = 0.5 * (ym[k] + yn[k] + hs * d[k]);
}

/* relative difference of two 3-vectors, on real parts (a decision) */
static double c_vrel(const cplx *a, const cplx *b) {
    double d0 = creal(a[0]) - creal(b[0]), d1 = creal(a[1]) - creal(b[1]),
           d2 = creal(a[2]) - creal(b[2]);
    double num = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    double den = sqrt(creal(a[0]) * creal(a[0]) + creal(a[1]) * creal(a[1]) +
                      creal(a[2]) * creal(a[2]));
    return den > 0.0 ? num / den : num;
}

static int c_bs_attempt(const c_ha_sys *s, const cplx *y0, double H, cplx *yout, cplx *T,
                        cplx *w) {
    int dim = 6 * s->ng;
    cplx *ym = w, *yn = w + dim, *d = w + 2 * dim, *tmp = w + 3 * dim;
#define TT(k, j) (&T[((size_t)(k) * CS_KMAX + (j)) * dim])
    for (int k = 0; k < CS_KMAX; ++k) {
        int nk = 2 * (k + 1);
        c_mmid(s, y0, H, nk, TT(k, 0), ym, yn, d, tmp);
        for (int j = 1; j <= k; ++j) {
            int nkj = 2 * (k - j + 1);
            double ratio = (double)nk / (double)nkj;
            double den = ratio * ratio - 1.0;
            cplx *cur = TT(k, j), *prev = TT(k, j - 1), *up = TT(k - 1, j - 1);
            for (int q = 0; q < dim; ++q) cur[q] = prev[q] + (prev[q] - up[q]) / den;
        }
        if (k >= 1) {
            double err = 0.0;
            const cplx *A = TT(k, k), *B = TT(k, k - 1);
            for (int i = 0; i < s->ng; ++i) {
                double ex = c_vrel(&A[6 * i], &B[6 * i]);
                double ev = c_vrel(&A[6 * i + 3], &B[6 * i + 3]);
                if (ex > err) err = ex;
                if (ev > err) err = ev;
            }
            if (err <= s->p->bs_tol) {
                memcpy(yout, A, sizeof(cplx) * dim);
                return 1;
            }
        }
    }
#undef TT
    return 0;
}

/* binary refinement over H, as bs_integrate2 without collisions */
static int c_bs_integrate(const c_ha_sys *s, cplx *y, double H, int64_t *substeps) {
    int dim = 6 * s->ng;
    int D = s->p->bs_max_depth;
    if (D < 0 || D > 40) return GO_EINVAL;
    cplx *T = (cplx *)malloc(sizeof(cplx) * dim * CS_KMAX * CS_KMAX);
    cplx *w = (cplx *)malloc(sizeof(cplx) * dim * 5);
    if (!T || !w) {
        free(T);
        free(w);
        return GO_EINVAL;
    }
    cplx *ynew = w + 4 * dim;
    int64_t pos = 0, total = (int64_t)1 << D;
    int d = 0;
    int rcode = GO_OK;
    while (pos < total) {
        double h = ldexp(H, -d);
        if (c_bs_attempt(s, y, h, ynew, T, w)) {
            memcpy(y, ynew, sizeof(cplx) * dim);
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

/* precheck on real parts, as genga_oracle.c */
static void c_precheck(const go_params *p, int n, const cplx *x, const cplx *rc, uint8_t *cand) {
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) cand[(size_t)i * n + j] = 0;
        for (int j = i + 1; j < n; ++j) {
            double d0 = creal(x[3 * j]) - creal(x[3 * i]),
                   d1 = creal(x[3 * j + 1]) - creal(x[3 * i + 1]),
                   d2 = creal(x[3 * j + 2]) - creal(x[3 * i + 2]);
            double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            double rcij = creal(rc[i]) > creal(rc[j]) ? creal(rc[i]) : creal(rc[j]);
            cand[(size_t)i * n + j] = r < p->pf * rcij;
        }
    }
}

/* One step of Eq. (7) with the step recipe of Sec. 2.2, as massive_step1 of
 * genga_oracle.c without collisions (candidates from the precheck). */
static int c_step(const go_params *p, int n, const cplx *m, cplx *x, cplx *v, cplx *rc,
                  uint8_t *cand, go_stats *st, cplx *acc, cplx *xm, cplx *vm, int32_t *pairs,
                  int32_t *label, int32_t *order, cplx *gy, cplx *gm, cplx *grc) {
    double h = 0.5 * p->dt;
    double mu = p->G * p->m0;
    if (p->encounter_free) {
        c_accel(p, n, m, x, rc, acc);
        for (int i = 0; i < 3 * n; ++i) v[i] += h * acc[i];
        c_sun_drift(p, n, m, x, v, h);
        for (int i = 0; i < n; ++i) {
            int it = 0;
            if (c_kepler(mu, C3(x, i), C3(v, i), p->dt, C3(x, i), C3(v, i), p->kepler_max_iter,
                         &it) != GO_OK)
                return GO_EKEPLER;
        }
        c_sun_drift(p, n, m, x, v, h);
        c_accel(p, n, m, x, rc, acc);
        for (int i = 0; i < 3 * n; ++i) v[i] += h * acc[i];
        return GO_OK;
    }
    /* 1 */
    c_rcrit(p, n, m, x, v, rc);
    /* 2, 3 */
    c_accel(p, n, m, x, rc, acc);
    for (int i = 0; i < 3 * n; ++i) v[i] += h * acc[i];
    c_sun_drift(p, n, m, x, v, h);
    /* 4 */
    memcpy(xm, x, sizeof(cplx) * 3 * n);
    memcpy(vm, v, sizeof(cplx) * 3 * n);
    for (int i = 0; i < n; ++i) {
        int it = 0;
        if (c_kepler(mu, C3(x, i), C3(v, i), p->dt, C3(x, i), C3(v, i), p->kepler_max_iter,
                     &it) != GO_OK)
            return GO_EKEPLER;
    }
    /* 5: encounters among the candidates (real parts) */
    int nenc = 0;
    for (int i = 0; i < n; ++i) {
        for (int j = i + 1; j < n; ++j) {
            double dx0[3], dv0[3], dx1[3], dv1[3];
            for (int k = 0; k < 3; ++k) {
                dx0[k] = creal(xm[3 * j + k]) - creal(xm[3 * i + k]);
                dv0[k] = creal(vm[3 * j + k]) - creal(vm[3 * i + k]);
                dx1[k] = creal(x[3 * j + k]) - creal(x[3 * i + k]);
                dv1[k] = creal(v[3 * j + k]) - creal(v[3 * i + k]);
            }
            double d2 = go_hermite_dmin2(p->dt, dx0, dv0, dx1, dv1);
            double rcij = creal(rc[i]) > creal(rc[j]) ? creal(rc[i]) : creal(rc[j]);
            if (d2 < rcij * rcij && cand[(size_t)i * n + j]) {
                pairs[2 * nenc] = i;
                pairs[2 * nenc + 1] = j;
                ++nenc;
            }
        }
    }
    st->n_enc = nenc;
    st->enc_total += nenc;
    st->n_groups = 0;
    st->max_group = 0;
    if (nenc > 0) {
        /* 6, 7 */
        st->n_groups = go_groups(n, nenc, pairs, label);
        for (int g = 0; g < n; ++g) {
            if (label[g] != g) continue;
            int ng = 0;
            for (int i = g; i < n; ++i)
                if (label[i] == g) order[ng++] = i;
            if (ng > st->max_group) st->max_group = ng;
            for (int q = 0; q < ng; ++q) {
                int i = order[q];
                for (int k = 0; k < 3; ++k) {
                    gy[6 * q + k] = xm[3 * i + k];
                    gy[6 * q + 3 + k] = vm[3 * i + k];
                }
                gm[q] = m[i];
                grc[q] = rc[i];
            }
            c_ha_sys s = {p, ng, gm, grc};
            int rc2 = c_bs_integrate(&s, gy, p->dt, &st->bs_substeps);
            if (rc2 != GO_OK) return rc2;
            for (int q = 0; q < ng; ++q) {
                int i = order[q];
                for (int k = 0; k < 3; ++k) {
                    x[3 * i + k] = gy[6 * q + k];
                    v[3 * i + k] = gy[6 * q + 3 + k];
                }
            }
        }
    }
    /* 8, 9 */
    c_sun_drift(p, n, m, x, v, h);
    c_accel(p, n, m, x, rc, acc);
    for (int i = 0; i < 3 * n; ++i) v[i] += h * acc[i];
    c_precheck(p, n, x, rc, cand);
    return GO_OK;
}

int go_cs_massive(const go_params *p, int n, const double *m, const double *x,
                  const double *v, const double *dm, const double *dx, const double *dv,
                  double hstep, int64_t nsteps, double *xT, double *vT, double *dxT,
                  double *dvT, go_stats *st) {
    if (n < 1 || nsteps < 0 || !(hstep > 0.0)) return GO_EINVAL;
    go_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    size_t N = (size_t)n;
    cplx *cm = (cplx *)malloc(sizeof(cplx) * N);
    cplx *cx = (cplx *)malloc(sizeof(cplx) * 3 * N);
    cplx *cv = (cplx *)malloc(sizeof(cplx) * 3 * N);
    cplx *rc = (cplx *)malloc(sizeof(cplx) * N);
    cplx *acc = (cplx *)malloc(sizeof(cplx) * 3 * N);
    cplx *xm = (cplx *)malloc(sizeof(cplx) * 3 * N);
    cplx *vm = (cplx *)malloc(sizeof(cplx) * 3 * N);
    cplx *gy = (cplx *)malloc(sizeof(cplx) * 6 * N);
    cplx *gm = (cplx *)malloc(sizeof(cplx) * N);
    cplx *grc = (cplx *)malloc(sizeof(cplx) * N);
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * (N * (N - 1) + 2));
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * N);
    uint8_t *cand = (uint8_t *)malloc(N * N);
    double *rcr = (double *)malloc(sizeof(double) * N);
    int rcode = GO_OK;
    if (!cm || !cx || !cv || !rc || !acc || !xm || !vm || !gy || !gm || !grc || !pairs ||
        !label || !order || !cand || !rcr) {
        rcode = GO_EINVAL;
    } else {
        for (size_t i = 0; i < N; ++i) cm[i] = CMPLX(m[i], hstep * (dm ? dm[i] : 0.0));
        for (size_t k = 0; k < 3 * N; ++k) {
            cx[k] = CMPLX(x[k], hstep * (dx ? dx[k] : 0.0));
            cv[k] = CMPLX(v[k], hstep * (dv ? dv[k] : 0.0));
        }
        /* the first step's candidates, as go_massive_init (real parts) */
        rcode = go_massive_init(p, n, m, x, v, rcr, cand);
        for (size_t i = 0; i < N; ++i) rc[i] = rcr[i];
        for (int64_t s = 0; s < nsteps && rcode == GO_OK; ++s) {
            rcode = c_step(p, n, cm, cx, cv, rc, cand, st, acc, xm, vm, pairs, label, order, gy,
                           gm, grc);
            if (rcode == GO_OK) ++st->steps;
        }
        for (size_t k = 0; k < 3 * N; ++k) {
            xT[k] = creal(cx[k]);
            vT[k] = creal(cv[k]);
            dxT[k] = cimag(cx[k]) / hstep;
            dvT[k] = cimag(cv[k]) / hstep;
        }
    }
    free(cm);
    free(cx);
    free(cv);
    free(rc);
    free(acc);
    free(xm);
    free(vm);
    free(gy);
    free(gm);
    free(grc);
    free(pairs);
    free(label);
    free(order);
    free(cand);
    free(rcr);
    return rcode;
}
