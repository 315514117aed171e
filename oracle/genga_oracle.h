/*
 * Plain FP64 CPU oracle for the hybrid symplectic N-body step of
 * Grimm & Stadel, "The GENGA Code" (arXiv:1404.2324).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a slow, obviously correct implementation written from the paper.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header or constant with the
 * GPU path.
 *
 * Conventions
 *   - Positions x are heliocentric, velocities v are barycentric
 *     ("democratic" coordinates, Sec. 2.1).  Arrays are n x 3 row-major.
 *   - Every routine is FP64 and is compiled with -ffp-contract=off.
 *   - Return codes: 0 ok, negative error (see GO_E*).
 */
#ifndef GENGA_ORACLE_H
#define GENGA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double G;          /* gravitational constant                            */
    double m0;         /* central mass                                      */
    double dt;         /* time step tau                                     */
    double n1, n2;     /* critical-radius factors, Eq. (6)                  */
    double pf;         /* prechecker enlargement of r_crit (3 in Sec. 2.2)  */
    double bs_tol;     /* Bulirsch-Stoer relative tolerance                 */
    int bs_max_depth;  /* max number of step halvings in BS                 */
    int kepler_max_iter;
    int encounter_free;/* 1: K == 1 everywhere (the MVS map of Sec. 2.1)    */
    int pad_;
} go_params;

typedef struct {
    int64_t steps;          /* steps taken by the last call              */
    int64_t n_cand;         /* |C|: precheck candidates entering the last step */
    int64_t n_enc;          /* |E and C|: encounters of the last step     */
    int64_t n_miss;         /* |E minus C|: encounters the precheck missed */
    int64_t n_groups;       /* groups of the last step                    */
    int64_t max_group;      /* largest group of the last step             */
    int64_t bs_substeps;    /* accepted BS substeps, summed over the call */
    int64_t enc_total;      /* encounters summed over the call            */
    int64_t miss_total;     /* precheck misses summed over the call       */
    int64_t kepler_iter_max;/* largest Kepler iteration count of the call */
    int64_t tp_enc;         /* test-particle encounters of the last step   */
    int64_t tp_enc_total;
    int64_t tp_removed;     /* test particles removed by collisions (call) */
} go_stats;

enum {
    GO_OK = 0,
    GO_EINVAL = -1,
    GO_EOVERFLOW = -3,
    GO_EKEPLER = -4,
    GO_EBS = -5,
    GO_EADJ_ENCOUNTER = -6
};

/* Threads of the OpenMP row loops (n > 0), and their current number. */
void go_set_threads(int n);
int go_threads(void);

/* ---- building blocks (exported for the pins) ---------------------------- */
void go_changeover(double y, double *K, double *dKdy);
void go_rcrit(const go_params *p, int n, const double *m, const double *x,
              const double *v, double *rc);
void go_accel(const go_params *p, int n, const double *m, const double *x,
              const double *rc, double *acc);
void go_sun_drift(const go_params *p, int n, const double *m, double *x,
                  const double *v, double h);
int go_kepler(double mu, const double *x0, const double *v0, double dt,
              double *x, double *v, int max_iter, int *iters);
void go_stumpff(double z, double c[4]);
int go_kepler_root(double mu, const double *x0, const double *v0, double dt, int max_iter,
                   double *s, int *iters);
double go_hermite_dmin2(double dt, const double *dx0, const double *dv0,
                        const double *dx1, const double *dv1);
int go_groups(int n, int npairs, const int32_t *ij, int32_t *label);
int go_bs_group(const go_params *p, int ng, const double *m, const double *rc,
                double *x, double *v, double H, int64_t *substeps);
void go_energy(const go_params *p, int n, const double *m, const double *x,
               const double *v, double *E, double *L);
void go_helio_to_dem(const go_params *p, int n, const double *m, double *v);
void go_dem_to_helio(const go_params *p, int n, const double *m, double *v);

/* ---- main mode ---------------------------------------------------------- */
int go_massive_init(const go_params *p, int n, const double *m,
                    const double *x, const double *v, double *rc,
                    uint8_t *cand);
int go_massive_step(const go_params *p, int n, const double *m, double *x,
                    double *v, double *rc, uint8_t *cand, int64_t nsteps,
                    go_stats *st, int enc_cap, int32_t *enc_ij,
                    double *enc_d2, double *enc_rc2, int *n_enc);

/* ---- complex-step derivative of the hybrid step (genga_cstep.c) ---------
 * nsteps steps of go_massive_step (no collisions) from (m, x, v) in complex
 * arithmetic along the direction (dm, dx, dv) (any may be NULL = 0) with
 * imaginary step hstep: xT, vT the real state (equal to go_massive_step's),
 * dxT, dvT the directional derivative of the state with every decision of
 * the run held fixed.  st: counters as go_massive_step (may be NULL).     */
int go_cs_massive(const go_params *p, int n, const double *m, const double *x,
                  const double *v, const double *dm, const double *dx, const double *dv,
                  double hstep, int64_t nsteps, double *xT, double *vT, double *dxT,
                  double *dvT, go_stats *st);

/* ---- higher orders (Sec. 2.3) ------------------------------------------- */
/* Sub-step coefficients of the composition of the given order (2, 4 or 6)
 * into w (up to 7); returns their number, 0 for another order.            */
int go_composition(int order, double *w);
/* nsteps composed steps (main mode): each sub-step w_k dt is the full hybrid
 * step with the encounter search over all pairs (no prechecker).  The
 * radii rc are those of the last sub-step on return.  st: counters summed
 * over the sub-steps (n_enc, n_groups, max_group: the last sub-step).     */
int go_massive_step_order(const go_params *p, int order, int n, const double *m, double *x,
                          double *v, double *rc, int64_t nsteps, go_stats *st);

/* ---- collisions and ejections of massive bodies (Sec. 3.2.7, 3.2.8, 3.4) */
enum { GO_EV_MERGE = 1, GO_EV_EJECT_FAR = 2, GO_EV_EJECT_SUN = 3 };
enum { GO_STOPPED = 2 };  /* fewer than nmin bodies left: the run stops */

typedef struct {
    int32_t kind;          /* GO_EV_*                                       */
    int32_t id_i, id_j;    /* merger: survivor and the absorbed body (their
                            * original indices); ejection: the body, -1     */
    int32_t pad_;
    int64_t step;          /* step index (step0 + steps of this call)       */
    double frac;           /* merger: part of the step before the colliding
                            * BS substep; ejection: 1                        */
    double m_i, m_j, R_i, R_j;
    double x_i[3], v_i[3], s_i[3];  /* democratic state and spin at the    */
    double x_j[3], v_j[3], s_j[3];  /* report (merger: start of the
                                     * colliding substep)                   */
    double U;              /* merger: internal energy, else 0              */
} go_event;

/* The main-mode step with collisions and ejections: *n bodies with radii R,
 * spins S (n x 3) and original indices id; m, x, v, rc, R, S, id change
 * as bodies merge or leave (the last body moves into each freed row, rows
 * in descending order, and *n shrinks).  rcut / rcut_sun: ejection limits on
 * the distance from the central mass (0 = off).  nmin: the run stops with
 * GO_STOPPED when fewer bodies remain.  Events go to ev (cap ev_cap; *n_ev
 * counts all, GO_EOVERFLOW when more than cap); *U accumulates the internal
 * energy of the mergers.  cand is the n x n candidate matrix of the current
 * n.  step0: steps taken before this call.                                 */
int go_massive_step_phys(const go_params *p, int *n, double *m, double *x, double *v,
                         double *rc, uint8_t *cand, int64_t nsteps, go_stats *st,
                         double *R, double *S, int32_t *id, double rcut, double rcut_sun,
                         int nmin, int64_t step0, go_event *ev, int ev_cap, int *n_ev,
                         double *U);
/* The merger of two bodies (Sec. 3.2.7): a perfectly inelastic merger that
 * conserves mass, momentum and angular momentum (orbital plus spin), with
 * the internal energy U = 1/2 m_i m_j/(m_i+m_j) v_ij^2 - G m_i m_j/r_ij.
 * y: x, v (6 values) per body; the merged body in m_out, y_out, R_out (the
 * radius of the merged volume), s_out; returns U.                          */
double go_merge(double G, double mi, double mj, const double *yi, const double *yj,
                double Ri, double Rj, const double *si, const double *sj, double *m_out,
                double *y_out, double *R_out, double *s_out);

/* ---- test-particle mode ------------------------------------------------- */
int go_tp_init(const go_params *p, int nm, const double *m, const double *x,
               const double *v, double *rc, uint8_t *cand, int64_t ntp,
               const double *xt, const double *vt, uint8_t *cand_tp);
/* rad: NULL (no collisions) or nm + ntp physical radii, planets first.
 * step0: steps taken before this call (for the collision reports).
 * A particle closer to a planet than the sum of their radii at any time of a
 * BS substep (Hermite interpolation over the substep, the encounter rule of
 * Sec. 2.2) is removed (Sec. 3.3): its report gets the planet index, the step
 * index, the fraction of the step at the start of that substep and the
 * particle's state there (democratic coordinates, x then v); xt and vt of a
 * removed particle become NaN and later steps skip it.  coll_planet holds -1
 * for particles still present.  The report arrays may be NULL when rad is.
 * tp_d2, tp_rc2: NULL (both), or ntp x nm arrays that receive, for the last
 * step of the call, the Hermite minimum squared separation (Eqs. 10-12) of
 * every particle-planet pair the prechecker had listed and its threshold
 * r_crit,ij^2; NaN for pairs not tested and for removed particles.  The
 * step's test-particle encounter set (Sec. 3.3) is {(k, j): d2 < rc2}. */
int go_tp_step(const go_params *p, int nm, const double *m, double *x,
               double *v, double *rc, uint8_t *cand, int64_t ntp, double *xt,
               double *vt, uint8_t *cand_tp, int64_t nsteps, go_stats *st,
               const double *rad, int64_t step0, int32_t *coll_planet,
               int64_t *coll_step, double *coll_frac, double *coll_xv,
               double *tp_d2, double *tp_rc2);

/* ---- encounter-free map, tangent-linear model and adjoint ---------------- */
int go_free_step(const go_params *p, int n, const double *m, double *x,
                 double *v, int64_t nsteps);
int go_free_tlm(const go_params *p, int n, const double *m, const double *x0,
                const double *v0, const double *dm, const double *dx0,
                const double *dv0, int64_t nsteps, double *xT, double *vT,
                double *dxT, double *dvT);
int go_free_adjoint(const go_params *p, int n, const double *m,
                    const double *x0, const double *v0, int64_t nsteps,
                    const double *gxT, const double *gvT, double *gx0,
                    double *gv0, double *gm);

#ifdef __cplusplus
}
#endif
#endif
