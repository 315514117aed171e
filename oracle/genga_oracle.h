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
 * for particles still present.  The report arrays may be NULL when rad is. */
int go_tp_step(const go_params *p, int nm, const double *m, double *x,
               double *v, double *rc, uint8_t *cand, int64_t ntp, double *xt,
               double *vt, uint8_t *cand_tp, int64_t nsteps, go_stats *st,
               const double *rad, int64_t step0, int32_t *coll_planet,
               int64_t *coll_step, double *coll_frac, double *coll_xv);

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
