/*
 * genga.h -- C ABI of the MI355X (gfx950) implementation of the hybrid
 * symplectic N-body step of Grimm & Stadel, "The GENGA Code: Gravitational
 * Encounters in N-body simulations with GPU Acceleration" (arXiv:1404.2324).
 *
 * The problem (Sec. 1, Sec. 3): bodies of mass m_i with positions x_i and
 * velocities v_i orbit a central mass m0.  One step of length tau is the
 * second-order composition of Eq. (7) of the Hamiltonian split Eqs. (1)-(3):
 * an opening kick of the perturbing part H_B (pair terms weighted by the
 * changeover function K of Eqs. 4-5), a Sun kick of H_C, a Kepler drift of
 * H_A (Eq. 9), the close-encounter search (Eqs. 10-12), grouping (App. A),
 * direct Bulirsch-Stoer integration of each group (Sec. 3.2.6), a second Sun
 * kick and a closing kick with the prechecker (Sec. 2.2).
 *
 * Conventions shared by every call
 *   - All floating point is IEEE double (FP64).
 *   - Position / velocity arrays are n x 3, row-major (x0 y0 z0 x1 ...).
 *   - "d_" pointers are device (HBM) pointers, "h_" pointers host pointers.
 *   - The caller owns all memory: state arrays, the workspace and outputs.
 *     The library owns only the opaque context; it never frees caller
 *     memory.  Device pointers handed to genga_init must outlive the context
 *     only when named so below (the workspace); state arrays are copied.
 *   - Work is enqueued on the caller's HIP stream (NULL = default stream).
 *     Only the calls documented as synchronising wait for the device.
 *   - Return value: GENGA_OK (0), or a negative GENGA_E* code.  Errors the
 *     device detects inside a step (non-convergence, overflow) are latched in
 *     a device status word and returned by the next synchronising call.
 */
#ifndef GENGA_H
#define GENGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct genga_ctx genga_ctx;

/* Integration parameters.  Defaults (genga_params_default) follow Sec. 2.1:
 * n1 = 3, n2 = 0.4; prechecker factor 3 (Sec. 2.2).  The Bulirsch-Stoer
 * tolerance, depth and the Kepler iteration cap are this library's choices. */
typedef struct genga_params {
    double G;               /* gravitational constant                      */
    double m0;              /* central mass (main and test-particle mode)  */
    double dt;              /* time step tau (may be negative)              */
    double n1, n2;          /* critical-radius factors of Eq. (6)          */
    double pf;              /* prechecker enlargement of r_crit             */
    double bs_tol;          /* BS relative tolerance per body               */
    int32_t bs_max_depth;   /* max halvings of a BS substep                 */
    int32_t kepler_max_iter;/* cap of the universal Kepler iteration        */
    int32_t encounter_free; /* 1: K == 1 (the MVS map); no encounter work   */
    int32_t cand_per_body;  /* candidate partners stored per body           */
    int32_t enc_cap;        /* capacity of the encounter list               */
    int32_t order;          /* 2 (or 0): the second-order step of Eq. (7);
                             * 4 or 6: Yoshida's composition of it (Sec. 2.3),
                             * main mode only                              */
    /* Ejections (Sec. 3.2.8) and the minimal body count (Sec. 3.4.6),
     * batched and main mode (main mode: second order with encounters;
     * test-particle mode: all 0): a body farther from its central mass
     * than rcut, or closer than rcut_sun, leaves the system (0 = no limit);
     * a system with fewer than nmin bodies left stops (0 = never).         */
    double rcut, rcut_sun;
    int32_t nmin;
    int32_t reserved;
} genga_params;

/* A merger or an ejection (Sec. 3.2.7, 3.2.8). */
enum { GENGA_EV_MERGE = 1, GENGA_EV_EJECT_FAR = 2, GENGA_EV_EJECT_SUN = 3 };
typedef struct genga_event_s {
    int32_t kind;           /* GENGA_EV_*                                     */
    int32_t sys;            /* the system (batched mode; 0 in main mode)       */
    int32_t id_i, id_j;     /* original rows: merger: the surviving and the
                             * absorbed body; ejection: the body and -1        */
    int64_t step;           /* the step (since init) in which it happened     */
    double frac;            /* merger: part of the step before the BS substep
                             * of the contact; ejection: 1                     */
    double m_i, m_j, R_i, R_j;        /* masses and physical radii             */
    double x_i[3], v_i[3], s_i[3];    /* democratic state and spin of each     */
    double x_j[3], v_j[3], s_j[3];    /* body at the report (merger: the start
                                       * of the substep of the contact)        */
    double U;               /* merger: the internal energy of Sec. 3.2.7      */
} genga_event;

/* Bins of the Kepler-iteration histogram in genga_stats_t. */
#define GENGA_KEPLER_BINS 16

typedef struct genga_stats_s {
    int64_t steps;          /* steps taken since init                       */
    int32_t n_cand;         /* candidate pairs entering the last step       */
    int32_t n_enc;          /* confirmed encounter pairs of the last step   */
    int32_t n_groups;       /* encounter groups of the last step            */
    int32_t max_group;      /* members of the largest group, last step      */
    int32_t kepler_iter_max;/* most Kepler iterations any drift needed      */
    int32_t tp_enc;         /* test-particle encounters of the last step    */
    int64_t bs_substeps;    /* accepted BS substeps since init              */
    int64_t enc_total;      /* encounters since init                        */
    int64_t full_kicks;     /* opening kicks that could not reuse the cache */
    int64_t tp_enc_total;
    int64_t tp_removed;     /* test particles removed by collisions         */
    uint32_t flags;         /* latched device error bits                    */
    uint32_t reserved;
    /* Kepler drifts since init by iteration count (Sec. 3.2.1: the f and g
     * iteration converges in a few steps): bin k < 15 counts the drifts of
     * the step that took k iterations, bin 15 those that took 15 or more or
     * did not converge.  Every body's drift of every step of genga_step
     * counts once (massive bodies, particles, every system of a batch). */
    int64_t kepler_hist[GENGA_KEPLER_BINS];
} genga_stats_t;

enum { GENGA_MASSIVE = 0, GENGA_TEST = 1, GENGA_BATCH = 2 };
enum { GENGA_HELIO = 0, GENGA_DEMOCRATIC = 1 };
enum {
    GENGA_OK = 0,
    GENGA_EINVAL = -1,      /* bad argument, NaN/Inf input, size limit      */
    GENGA_EHIP = -2,        /* a HIP runtime call failed                    */
    GENGA_EOVERFLOW = -3,   /* candidate / encounter list capacity exceeded */
    GENGA_EKEPLER = -4,     /* universal Kepler iteration did not converge  */
    GENGA_EBS = -5,         /* Bulirsch-Stoer depth exhausted               */
    GENGA_EADJ_ENCOUNTER = -6, /* pair inside r_crit in the K = 1 adjoint map */
    GENGA_ENOMEM = -7,      /* workspace smaller than genga_workspace_bytes */
    GENGA_EGROUP = -8,      /* encounter group larger than supported        */
    GENGA_WSTOPPED = 1,     /* warning, batched mode: some systems stopped   */
    GENGA_WNMIN = 2         /* batched system status: fewer than nmin bodies  */
};

/* Fill *p with the defaults: G = 1, m0 = 1, dt = 2 pi / 100, n1 = 3,
 * n2 = 0.4 (Sec. 2.1), pf = 3 (Sec. 2.2), bs_tol = 1e-13, bs_max_depth =
 * 20, kepler_max_iter = 40, encounter_free = 0, cand_per_body = 32,
 * enc_cap = 16384, order = 2.  The encounter list may hold any number of
 * pairs (enc_cap); the grouping keeps the first 2048 in LDS and reads the
 * rest from the list. */
void genga_params_default(genga_params *p);

/* Device workspace (bytes) a context of this shape needs.  Main mode:
 * n_massive <= 2048 bodies with encounters (the paper's main-mode limit,
 * Sec. 3), <= 65536 with encounter_free, n_test = 0.  Test-particle mode:
 * 1 <= n_massive <= 32 (Sec. 3.3), 0 <= n_test <= 2^30.  Batched mode:
 * 1 <= n_sys <= 2^24 systems of 1..64 bodies, n_bodies in all (n_massive and
 * n_test unused).  Returns 0 for an unsupported shape or invalid parameters. */
size_t genga_workspace_bytes(int mode, const genga_params *p, int n_massive,
                             int64_t n_test, int n_sys, int64_t n_bodies);

/* Create a context and load the initial state (Sec. 2.2: the first opening
 * kick is prepared here, from the initial positions).
 *   mode        GENGA_MASSIVE (main mode), GENGA_TEST (test-particle mode,
 *               Sec. 3.3: n_massive bodies take the main-mode step and n_test
 *               massless particles feel them, but nothing else) or
 *               GENGA_BATCH (Sec. 3.4: n_sys independent systems, each with
 *               its own central mass; system s holds rows
 *               [d_offsets[s], d_offsets[s+1]) of every array).
 *   d_offsets   batched mode: n_sys + 1 int32 (device, read once): 0, then
 *               increasing, each system 1..64 bodies.
 *   d_m0        batched mode: n_sys central masses (device, read once), or
 *               NULL for p->m0 everywhere.
 *   d_m         n_massive masses (device, read once).
 *   d_x, d_v    (n_massive + n_test) x 3 positions and velocities (device,
 *               read once): the massive bodies' rows first, then the
 *               particles'.  coords_in = GENGA_HELIO: heliocentric positions
 *               and velocities, converted to democratic coordinates
 *               (heliocentric positions, barycentric velocities, Sec. 2.1,
 *               with the massive bodies' momentum); GENGA_DEMOCRATIC:
 *               already democratic.  A particle row of six NaN is a removed
 *               particle.
 *   d_workspace at least genga_workspace_bytes bytes of device memory, 256-B
 *               aligned, owned by the caller, used until genga_destroy.
 *   stream      hipStream_t of the caller (NULL = default stream).
 * Synchronises (validation of the input; batched mode also runs the tuner
 * of genga_tune for 4 steps on a copy of the state).  Errors: EINVAL (shape,
 * NaN or Inf in the input, non-positive m0, bad offsets), ENOMEM (workspace
 * too small), EHIP.  n_sys, d_offsets, d_m0 are for the batched mode only;
 * pass 0 / NULL otherwise; n_massive and n_test are 0 in batched mode. */
int genga_init(genga_ctx **ctx, int mode, const genga_params *p,
               int n_massive, int64_t n_test, int n_sys,
               const int32_t *d_offsets, const double *d_m0,
               const double *d_m, const double *d_x, const double *d_v,
               int coords_in, void *d_workspace, size_t ws_bytes,
               void *stream);

/* Advance nsteps steps of Eq. (7), following the step recipe of Sec. 2.2:
 * opening kick (reusing the closing kick's accelerations for non-candidate
 * pairs, Sec. 3.2.3), Sun kick, Kepler drift, encounter search, grouping,
 * BS integration of groups, Sun kick, closing kick with the prechecker.
 * With order 4 or 6 each step is Yoshida's composition of that step (Sec.
 * 2.3: sub-steps w_k dt, some backward in time; fourth order w1, w0, w1 with
 * w1 = 1/(2 - 2^(1/3)); sixth order his solution A), every sub-step the full
 * scheme with its own critical radii and the encounter search over all
 * pairs in place of the prechecker's candidates.
 * Asynchronous on the context's stream (replays a captured HIP graph);
 * errors latch in the device status.  nsteps >= 0. */
int genga_step(genga_ctx *ctx, int64_t nsteps);

/* Measurement form of genga_step (second order only): the same nsteps
 * (1..4096) steps launched
 * one kernel at a time (no graph) on the context's stream, back to back, the
 * closing-kick pair kernel through hipExtLaunchKernel with two HIP events
 * that take its dispatch's start and end timestamps; *h_kick_us receives
 * that kernel's average duration in microseconds.  Synchronising; returns
 * the latched status. */
int genga_step_profiled(genga_ctx *ctx, int64_t nsteps, double *h_kick_us);

/* Number of kernels of one main-mode step, and their order. */
#define GENGA_STEP_KERNELS 5
/* Run nsteps (1..512) main-mode steps (in test-particle mode followed by the
 * particle kernels, untimed) with a HIP event pair around every kernel of
 * the step, launched so that the events take the dispatch's own start and
 * end timestamps.  h_us[GENGA_STEP_KERNELS] (host, caller-owned) receives
 * each kernel's average duration in microseconds, in launch order: opening
 * kick with Sun kick and Kepler drift, encounter search (Eqs. 10-12),
 * grouping (App. A) with Bulirsch-Stoer of the groups (Sec. 3.2.6) in one
 * kernel, pair kernel of the closing kick (partial sums with the
 * prechecker), the closing kick's per-body epilogue (the partial sums
 * added, second Sun kick, velocity update, next critical radii); the second
 * and third are 0 with encounter_free.  The
 * breakdown behind a step's time, not a faster step.  Synchronising; returns
 * the latched status (GENGA_EINVAL for a batched context, a null pointer or
 * nsteps out of range). */
int genga_step_kernel_us(genga_ctx *ctx, int64_t nsteps, double *h_us);

/* Wait for the context's stream and return the latched device status as a
 * GENGA_E* code (GENGA_OK when clean).  Synchronising. */
int genga_sync(genga_ctx *ctx);

/* Write the current state to d_x, d_v (n x 3, device, caller-owned) in
 * GENGA_HELIO or GENGA_DEMOCRATIC coordinates.  Synchronising; returns the
 * latched status. */
int genga_get_state(genga_ctx *ctx, double *d_x, double *d_v, int coords_out);

/* Replace the state (same shape) and prepare the next opening kick as
 * genga_init does.  Synchronising. */
int genga_set_state(genga_ctx *ctx, const double *d_x, const double *d_v,
                    int coords_in);

/* Batched mode: replace the mass of every row (d_m, n_bodies doubles,
 * device) keeping positions and velocities, then prepare the next opening
 * kick as genga_init does (the masses enter Eqs. 1-3 and 6).  With
 * genga_set_state in democratic coordinates this re-runs a context from new
 * initial conditions without a new init.  Synchronising.  Errors: EINVAL
 * (other mode, NULL, a non-finite mass), EHIP. */
int genga_set_masses(genga_ctx *ctx, const double *d_m);

/* Total energy E = H_A + H_B + H_C of Eqs. (1)-(3) (K summed out:
 * sum m v^2/2 + |P|^2/2m0 - sum G m0 m_i/r_i - sum_{i<j} G m_i m_j/r_ij) and
 * angular momentum L = sum m_i x_i x v_i of each system, written to d_E
 * (n_sys doubles) and d_L (3 n_sys doubles), device, asynchronous.  The
 * relative energy error of Sec. 4.1 is |(E_t - E_0)/E_0|. */
int genga_energy(genga_ctx *ctx, double *d_E, double *d_L);

/* H_B acceleration (the kick's pair sum, Sec. 3.2.3) of the current state
 * with this step's critical radii, written to d_acc (n x 3, device).  Only
 * the pair kernel runs; the state is not changed.  Asynchronous. */
int genga_accel_state(genga_ctx *ctx, double *d_acc);

/* Confirmed close-encounter pairs of the last step (the Encounter kernel
 * output, Sec. 3.2.4): i < j body indices in h_ij (2 per pair; rows of the
 * whole state in batched mode), the Hermite minimum squared separation in
 * h_dmin2 and r_crit,ij^2 in h_rc2 (either may be NULL; NaN in batched
 * mode), sorted by (i, j).  *h_n receives the count; if it exceeds cap,
 * cap pairs are written and GENGA_EOVERFLOW is returned.  Synchronising. */
int genga_encounters(genga_ctx *ctx, int32_t *h_ij, double *h_dmin2,
                     double *h_rc2, int cap, int *h_n);

/* Prechecker candidates entering the next step (Sec. 2.2): pairs i < j with
 * r_ij < pf r_crit,ij at the end of the last closing kick, sorted, as in
 * genga_encounters.  h_r2 (may be NULL) receives r_ij^2 as the closing kick
 * computed it (NaN in batched mode, whose kernel keeps only the pair bits).
 * Synchronising. */
int genga_candidates(genga_ctx *ctx, int32_t *h_ij, double *h_r2, int cap, int *h_n);

/* Test-particle mode: the particle-planet close encounters of the last step
 * (Sec. 3.3: a particle that meets a planet within the critical radius is
 * integrated with it by BS; the set is the prechecker's candidates whose
 * Hermite minimum of Eqs. 10-12 falls below r_crit,ij^2).  Per pair: particle
 * index among the particles (h_tp), massive-body index (h_planet), the
 * Hermite minimum squared separation (h_d2) and r_crit,ij^2 (h_rc2), as the
 * step's kernel computed them (copied, no arithmetic); sorted by (particle,
 * planet).  Particles removed in that step keep their encounter there.  Host
 * arrays of cap entries (h_d2, h_rc2 may be NULL); *h_n receives the count;
 * GENGA_EOVERFLOW when it exceeds cap (cap pairs written).  Synchronising.
 * Errors: EINVAL (other mode). */
int genga_tp_encounters(genga_ctx *ctx, int64_t *h_tp, int32_t *h_planet, double *h_d2,
                        double *h_rc2, int64_t cap, int64_t *h_n);

/* Physical radii (Sec. 3.2.7), device array, copied.  Batched mode and main
 * mode (second order, with encounters): one per row; any positive radius
 * turns on the mergers described at genga_events.
 * Test-particle mode (Sec. 3.3): n_massive + n_test values (planets first).
 * From the next step on,
 * a particle whose separation from a planet, Hermite-interpolated over a
 * Bulirsch-Stoer substep of its encounter (Eqs. 10-12 over that substep),
 * falls below the sum of their radii is removed: its x and v become NaN,
 * later steps skip it, and a report is kept (genga_collisions).  Radii start
 * at 0 (no collisions).  A particle only meets this test inside an encounter,
 * so radii should stay below the critical radii.  Synchronising.  Errors:
 * EINVAL (main mode with composed steps or encounter_free, negative or
 * non-finite radius; test-particle radii are then reset to 0, main-mode and
 * batched radii left as they were), EHIP. */
int genga_set_radii(genga_ctx *ctx, const double *d_radii);

/* Reports of the particles removed since init, sorted by (step, particle):
 * particle index among the particles (h_tp), massive-body index (h_planet),
 * step index since init (h_step), part of that step covered before the BS
 * substep of the collision (h_frac, a multiple of 2^-bs_max_depth), and the
 * particle's democratic state at the start of that substep (h_xv, 6 per
 * report: x then v).  Host arrays of cap entries; *h_n receives the count;
 * GENGA_EOVERFLOW when it exceeds cap (cap reports written).  Synchronising. */
int genga_collisions(genga_ctx *ctx, int64_t *h_tp, int32_t *h_planet,
                     int64_t *h_step, double *h_frac, double *h_xv,
                     int64_t cap, int64_t *h_n);

/* Batched mode: time each kernel variant (register budget per wave: 1, 2 or
 * 4 waves per SIMD; one system per wave handed out in index order or
 * largest first, or two systems per wave, consecutive in the largest-first
 * order, for systems of up to 32 bodies) for nsteps steps on a copy of the
 * current state, with HIP events on the context's stream, and keep the
 * fastest for later steps.  All variants give the same results.  h_us (host,
 * cap doubles) receives each variant's time in microseconds (-1 for a
 * variant these systems cannot use: two per wave with a system over 32
 * bodies), *h_n the number of variants (9), *h_choice the variant kept.  The
 * state is not advanced.  Synchronising.  Errors: EINVAL (other mode),
 * EOVERFLOW (cap < 9), EHIP. */
int genga_tune(genga_ctx *ctx, int nsteps, double *h_us, int cap, int *h_n,
               int *h_choice);

/* Description of tuner variant v (static storage; "?" outside 0..8). */
const char *genga_tune_variant(int v);

/* Batched mode: use variant v (as numbered by genga_tune) for later steps
 * instead of the tuner's choice.  Not synchronising.  Errors: EINVAL (other
 * mode, v outside 0..8, or a two-systems-per-wave variant with a system over
 * 32 bodies). */
int genga_batch_set_variant(genga_ctx *ctx, int v);

/* Batched mode: a system whose step fails (Kepler non-convergence, BS depth)
 * stops there with the state it had before that step, and the others go on
 * (the paper's multi-simulation mode stops systems individually, Sec. 3.4);
 * the synchronising calls then return the warning GENGA_WSTOPPED.  Per
 * system (host arrays of cap entries): h_status the error that stopped it
 * (GENGA_OK while running), h_steps the steps it completed since init.
 * Synchronising.  Errors: EINVAL (other mode), EOVERFLOW (cap < n_sys). */
int genga_batch_status(genga_ctx *ctx, int32_t *h_status, int64_t *h_steps,
                       int cap);

/* Collisions and ejections (Sec. 3.2.7, 3.2.8, 3.4.6), batched mode and
 * main mode (second order with encounters; a main-mode run is one system,
 * sys = 0).  With physical radii set (genga_set_radii, one per row) two
 * bodies of a group of up to 64 members (GENGA_EGROUP for larger groups
 * with radii)
 * that come closer than the sum of their radii during a BS substep (the
 * Hermite test of Eqs. 10-12 applied to the substep) merge at the start of
 * that substep: mass, momentum and orbital-plus-spin angular momentum are
 * kept, the radius is that of the summed volume, the more massive body
 * survives (the lower row on equal masses), and the group is integrated
 * over the rest of the step.  With rcut / rcut_sun (genga_params) bodies
 * beyond or inside those distances from their central mass leave after the
 * direct integration.  Each freed row takes the system's last body (freed
 * rows in descending order) and the system's count drops; with fewer than
 * nmin bodies left a system stops (status GENGA_WNMIN; in main mode the
 * synchronising calls return that warning and later steps change nothing).
 * genga_get_state writes NaN rows past a system's count.
 * genga_events: every merger and ejection since init (host array of cap
 * records), sorted by (step, system, part of the step, survivor); *h_n
 * receives the count, GENGA_EOVERFLOW when it exceeds cap or the record
 * store (one record per row).  Synchronising.  Errors: EINVAL
 * (test-particle mode).
 * genga_bodies: per row the original row of the body it holds (-1 past the
 * system's count; host, cap >= the rows), per system the bodies left and
 * the summed internal energy U of its mergers (host, sys_cap >= n_sys).
 * Synchronising.  Errors: EINVAL (test-particle mode), EOVERFLOW (small
 * caps). */
int genga_events(genga_ctx *ctx, genga_event *h_ev, int64_t cap, int64_t *h_n);
int genga_bodies(genga_ctx *ctx, int32_t *h_id, int64_t cap, int32_t *h_nlive, double *h_U,
                 int sys_cap);

/* ---- reverse-mode gradients ------------------------------------------------
 * The paper has no adjoint.  Two maps of a batched context are
 * differentiated, chosen by its parameters:
 *  - encounter_free = 1: the map with K = 1 (the MVS map in democratic
 *    coordinates, Sec. 2.1; kick tau/2, Sun kick tau/2, Kepler drift tau,
 *    Sun kick tau/2, kick tau/2), exactly (up to rounding);
 *  - encounter_free = 0, no radii, rcut = rcut_sun = 0: the second-order
 *    hybrid step (Eq. 7, Sec. 2.2) with the changeover K, K' (Eqs. 4-5), the
 *    critical radii (Eq. 6) as functions of the state and masses, the
 *    encounter test (Eqs. 10-12), the groups (App. A) and BS of H_A per
 *    group, differentiated with every decision of the run held fixed
 *    (candidates, encounters, groups, accepted BS substeps and their
 *    extrapolation column, branches of K and Eq. 6).  The first step's
 *    candidates are the precheck of the initial state with its own radii.
 *    A group that takes more than 64 accepted BS substeps in one step
 *    latches GENGA_EOVERFLOW in the backward pass; BS depth exhaustion
 *    GENGA_EBS. */

/* Bytes of the caller's buffer for nsteps steps with a checkpoint every
 * ckpt_every steps (the checkpoints plus the backward pass's workspace: one
 * segment's tape, and for the hybrid map the starts of a group's accepted BS
 * substeps and the positions of one Gragg sequence); 0 when the context
 * supports neither map or the arguments are invalid. */
size_t genga_adj_buffer_bytes(genga_ctx *ctx, int64_t nsteps, int ckpt_every);

/* Advance every system nsteps steps of the context's map, keeping the state
 * (and for the hybrid map the candidate set) every ckpt_every steps in
 * d_buffer (device, 256-B aligned, caller-owned, at least
 * genga_adj_buffer_bytes; it must stay untouched until the matching
 * genga_adj_backward).  Asynchronous.  Encounter-free map: a pair that comes
 * inside its critical radius (Eq. 6) latches GENGA_EADJ_ENCOUNTER (the
 * hybrid method would no longer use K = 1 there).  Errors: EINVAL, ENOMEM,
 * EHIP. */
int genga_adj_forward(genga_ctx *ctx, int64_t nsteps, int ckpt_every,
                      void *d_buffer, size_t buffer_bytes);

/* Gradients through the last genga_adj_forward: given dL/dx_T and dL/dv_T
 * (device, rows x 3, democratic coordinates) write dL/dx_0, dL/dv_0 (rows x
 * 3) and dL/dm (rows) of the state before it.  Recomputes each segment from
 * its checkpoint (the state is not changed).  Asynchronous. */
int genga_adj_backward(genga_ctx *ctx, const double *d_gxT, const double *d_gvT,
                       double *d_gx0, double *d_gv0, double *d_gm);

/* Counters of the run (h_stats host).  Synchronising. */
int genga_stats(genga_ctx *ctx, genga_stats_t *h_stats);

/* Message for a GENGA_E* code (static storage). */
const char *genga_strerror(int code);

/* Release the context (not the caller's memory).  Synchronising. */
int genga_destroy(genga_ctx *ctx);

/* ---- component operations (same kernels' building blocks) ------------- */

/* Acceleration of the perturbing part H_B (the kick of Eq. 7, Sec. 3.2.3):
 * a_i = sum_{j != i} G m_j [K/r^3 - K'(r)/r^2] (x_j - x_i) with
 * r_crit,ij = max(d_rc[i], d_rc[j]); encounter_free gives K = 1.
 * d_m (n), d_x (n x 3), d_rc (n) in; d_acc (n x 3) out; all device.
 * Uses the context-free workspace of genga_accel_workspace_bytes(n).
 * Asynchronous.  Errors: EINVAL, ENOMEM, EHIP. */
size_t genga_accel_workspace_bytes(int n);
int genga_accel(const genga_params *p, int n, const double *d_m,
                const double *d_x, const double *d_rc, double *d_acc,
                void *d_workspace, size_t ws_bytes, void *stream);

/* genga_accel with no workspace argument and no allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, same
 * kernels and the same bits as genga_accel, for 1 <= n <=
 * GENGA_ACCEL_NOALLOC_MAX bodies (EINVAL beyond).  The library keeps the
 * packed bodies, radii and thresholds in a fixed device array of its own,
 * about 5.0 MB, one per GPU, held until the process ends; the first call on
 * a device looks up that device's copy (on the device current at the call,
 * which must be the stream's).  Calls that overlap on one GPU (concurrent
 * streams or threads) share that array and race: serialise them.
 * Asynchronous.  Errors: EINVAL, EHIP. */
#define GENGA_ACCEL_NOALLOC_MAX 16384
int genga_accel_noalloc(const genga_params *p, int n, const double *d_m,
                        const double *d_x, const double *d_rc, double *d_acc,
                        void *stream);

/* Kepler drift of n independent bodies for dt about mu (Eq. 9, universal
 * variables).  d_x0, d_v0 in, d_x, d_v out (n x 3, device; may alias the
 * inputs).  d_iters (n ints, device, may be NULL) receives the iteration
 * count, negative when the iteration did not converge.  Asynchronous. */
int genga_kepler(double mu, int64_t n, const double *d_x0, const double *d_v0,
                 double dt, double *d_x, double *d_v, int max_iter,
                 int32_t *d_iters, void *stream);

/* Hermite close-encounter minimum of Eqs. (10)-(12) for n pairs.  d_q holds
 * 12 doubles per pair (dx0, dv0, dx1, dv1: relative position and velocity at
 * the start and the end of the step); d_out receives the minimum squared
 * separation per pair.  Device pointers, asynchronous. */
int genga_hermite(int64_t n, double dt, const double *d_q, double *d_out,
                  void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GENGA_H */
