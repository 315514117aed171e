// Internal declarations of the GENGA MI355X library: device-resident status
// words, the per-mode workspace views and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/genga.h"

namespace genga {

// latched error bits of the device status word
enum : unsigned {
  F_KEPLER = 1u,       // Kepler iteration did not converge
  F_BS = 2u,           // Bulirsch-Stoer depth exhausted
  F_CAND_OVF = 4u,     // per-body candidate table full
  F_ENC_OVF = 8u,      // encounter list full
  F_GROUP = 16u,       // group larger than the in-wave BS limit
  F_TP_OVF = 32u,      // more massive bodies than the test-particle mask holds
  F_ADJ_ENC = 64u,     // a pair inside r_crit during the encounter-free map
  F_SYS_STOP = 128u,   // batched: a system stopped after a failed step (warning)
  F_NMIN = 256u,       // batched: a system stopped with fewer than nmin bodies
  F_ADJ_LEAF = 512u,   // hybrid adjoint: a group took more BS substeps in a step than it keeps
};
// control bits
enum : unsigned { C_FULLKICK = 1u };

struct DevStat {
  unsigned flags;      // latched errors
  unsigned ctl;        // control bits, consumed inside a step
  int nenc;            // confirmed encounters of the last step
  int ngroups;         // groups of the last step
  int maxg;            // largest group of the last step
  int ncand;           // candidate pairs (i<j) entering the last step
  int kep_itmax;       // largest Kepler iteration count seen
  unsigned long long bs_sub;     // accepted BS substeps (cumulative)
  unsigned long long enc_total;  // encounters (cumulative)
  unsigned long long fullkicks;  // opening kicks recomputed in full
  unsigned long long nstep;      // steps begun since init
  unsigned long long tp_removed; // test particles removed by collisions
  double P2[4];        // momentum for the second Sun kick of the step
  int nlive;           // main mode: bodies present (rows past it are padding)
  int stopped;         // main mode: fewer than nmin bodies left, steps do nothing
  double U;            // main mode: summed internal energy of the mergers
  unsigned long long ev_cnt;  // main mode: mergers and ejections since init
  double Pej[4];       // main mode: momentum of the bodies ejected in the step
};

// Report of a test particle removed by a collision with a planet.
struct CollRec {
  long long tp;        // particle index (0-based among the particles)
  long long step;      // step index since init
  int planet;          // massive-body index
  int pad;
  double frac;         // part of the step covered before the colliding substep
  double xv[6];        // the particle's democratic state there
};

constexpr int kKepBins = GENGA_KEPLER_BINS;  // Kepler-iteration histogram bins
constexpr int kBsMaxGroup = 64;        // members of the lane-per-member BS path
constexpr int kGroupMaxN = 2048;       // bodies the one-workgroup grouping holds
constexpr int kEncLds = 2048;          // encounter pairs grouped in LDS
constexpr int kVecBlock = 256;         // threads of the per-body kernels
constexpr int kOpenBlock = 64;         // threads of the opening-kick-and-drift kernel (one wave)

// Views into the caller's workspace for main mode (also the massive part of
// test-particle mode).  Bodies are padded to np (a multiple of 256).
struct MassiveWs {
  int n, np, njs, pw, nblk;        // njs: partner splits of the pair kernel, pw: its waves per workgroup
  int cpb;              // candidate slots per body
  int enc_cap;
  double4* xm;          // x, y, z, m          (democratic: heliocentric x)
  double4* vv;          // vx, vy, vz, 0       (barycentric v)
  double4* xs;          // x, m between steps (the closing kick's output; the
                        // opening kick reads its partners here)
  double4* xpre;        // pre-drift x
  double4* vpre;        // pre-drift v
  double4* afar;        // acceleration of non-candidate pairs (x G)
  double* rc_cur;       // radii of the current step
  double* rc_next;      // radii for the next step
  double* thr;          // max((pf rc)^2, tiny): candidate threshold
  double* tmax64;       // largest threshold of each 64-body chunk [np/64]
  double* pp;           // pair kernel's partial sums [njs][6][np]
  double* partP;        // momentum partials after the opening kick [nblk][4]
  double* partP2;       // momentum partials after the drift [nblk][4]
  double* dP;           // momentum change of each BS group [np/2+1][4]
  double* red;          // scratch for reductions (energy, conversions)
  int* ccnt;            // candidates per body
  int* ctab;            // candidate partners [np][cpb]
  double* cr2;          // their squared separations [np][cpb]
  unsigned long long* khist;  // Kepler iterations per block, cumulative [nblk][kKepBins]
  int2* encij;          // encounter pairs of the last step
  double* encd2;
  double* encrc2;
  int* goff;            // group offsets [np+1]
  int* gmem;            // group members [np]
  double* rad;          // physical radii (collisions, Sec. 3.2.7) [np]
  double4* sp;          // spins [np]
  int* ids;             // original row of the body in each row [np]
  int* dead;            // bodies leaving in this step [np]
  genga_event* ev;      // mergers and ejections since init [ev_cap]
  int ev_cap;
  double* bsbig;        // BS records of members of groups over 64 [np][66]
  double4* bspos;       // their Gragg-point positions and masses [np]
  int* bsmem;           // their sorted member lists (at the group offsets) [np]
  int* flag_in;         // input validation flag
  double4* xstart;      // positions at the start of the step (test-particle mode)
  double4* xpost;       // state after the drift, before BS (test-particle mode)
  double4* vpost;
  DevStat* st;
};

// Test-particle state and the per-step list of particles needing BS.
struct TpWs {
  int64_t ntp;
  double* x;            // [3][ntp]
  double* v;            // [3][ntp]
  unsigned* mask;       // candidate planets per particle
  int* bs_idx;          // listed particles
  unsigned* bs_mask;    // their encounter planets (cleared as they finish)
  unsigned* bs_emask;   // the same, kept for the encounter report
  double* enc_d2;       // Hermite minimum of each encounter [nm][ntp]
  double* enc_rc2;      // its threshold r_crit,ij^2 [nm][ntp]
  int nm;               // massive bodies (stride of enc_d2, enc_rc2)
  double* bs_rct;       // their critical radii
  double* bs_y;         // their pre-drift state [6][ntp]
  double* rad;          // physical radii: planets [32], then particles [ntp]
  CollRec* coll;        // collision reports, one slot per particle
  int64_t nb, cap;      // 256-particle blocks; list capacity nb * 256
  int* blk_cnt;         // listed particles per block (this step)
  int* blk_off;         // their prefix sum [nb + 1]
  int* blk_enc;         // encounters per block (this step)
  unsigned long long* blk_enc_tot;  // encounters per block since init
  int* blk_kit;         // largest Kepler iteration count per block
  unsigned long long* khist;  // Kepler iterations per block, cumulative [nb][kKepBins]
  unsigned long long* sub;          // accepted BS substeps per workgroup / wave
  double* pl;           // planets' whole-step BS table
  int64_t* rq;          // listed entries left to the wave path (this step)
  int* rq_cnt;          // their count
  void* cum;            // the cumulative counters above, cleared at init
  size_t cum_bytes;
};

constexpr int kTpMaxPlanets = 32;
constexpr int kTpBs1Grid = 1024;   // workgroups of the whole-step BS attempt
constexpr int kTpBsGrid = 2048;    // waves of the refinement path
constexpr int kTpSubSlots = kTpBs1Grid + kTpBsGrid;

struct TpCounters {
  long long enc;                 // encounters of the last step
  unsigned long long enc_total;  // since init
  int kit;                       // largest Kepler iteration count
  unsigned long long sub;        // accepted BS substeps since init
  unsigned long long khist[kKepBins];  // Kepler iterations since init
};

struct StepConsts {
  double G, m0, mu, dt, h, n1, n2, pf, pf2, bs_tol;
  int bs_max_depth, kepler_max_iter, encounter_free;
  // composed steps (Sec. 2.3): |dt| of the sub-step that follows (its
  // critical radii are formed at the end of this one), and the encounter
  // search over every pair instead of the prechecker's candidates
  double absdt_next;
  int all_pairs;
  // bodies can leave (Sec. 3.2.7, 3.2.8, 3.4.6): phys adds the compaction
  // after BS, coll the collision tests inside BS (some radius positive)
  int phys, coll, nmin;
  double rcut, rcut_sun;
};

// Sub-steps of the composed step of the given order (2: one, 4: three, 6:
// seven), their coefficients in w; 0 for an unsupported order.
int composition(int order, double* w);

StepConsts make_consts(const genga_params& p);
// Finite parameters inside their documented ranges.
bool params_valid(const genga_params* p);

// ---- main-mode launchers (massive.hip) --------------------------------------
size_t massive_ws_bytes(int n, const genga_params& p, bool snap = false);
size_t massive_carve(MassiveWs& w, int n, const genga_params& p, void* base,
                     bool snap = false);
hipError_t validate_finite(const double* a, int64_t cnt, int* dbad,
                           hipStream_t s);
hipError_t massive_pack(const MassiveWs& w, const StepConsts& c,
                        const double* m, const double* x, const double* v,
                        int coords_in, hipStream_t s);
hipError_t massive_unpack(const MassiveWs& w, const StepConsts& c, double* x,
                          double* v, int coords_out, hipStream_t s);
hipError_t massive_prime(const MassiveWs& w, const StepConsts& c,
                         hipStream_t s);
// Every body present in its own row (count, original rows, spins; radii too
// with clear_radii).
hipError_t massive_reset_bodies(const MassiveWs& w, bool clear_radii, hipStream_t s);
// Kernels of one main-mode step in launch order: opening kick and drift,
// encounter search, grouping with BS, pair kernel (partial sums), the
// closing kick's per-body epilogue (the second and third only with
// encounters).  With
// kev (2 kStepKernels events), the events of slot k take the start and end
// timestamps of kernel k's dispatch.
constexpr int kStepKernels = 5;
constexpr int kSlotPairs = 3;  // the pair kernel's slot
hipError_t massive_step(const MassiveWs& w, const StepConsts& c, hipStream_t s,
                        const hipEvent_t* kev = nullptr);
hipError_t massive_energy(const MassiveWs& w, const StepConsts& c, double* dE,
                          double* dL, hipStream_t s);
// H_B acceleration of positions x (w = mass; x = xs for a context's state).
hipError_t massive_accel(const MassiveWs& w, const StepConsts& c, const double4* x,
                         double* acc, hipStream_t s);
hipError_t thresholds_from_radii(const MassiveWs& w, const StepConsts& c,
                                 hipStream_t s);
hipError_t massive_masses(const MassiveWs& w, double* m, hipStream_t s);
// H_B acceleration of n bodies given as caller arrays (m, x n x 3, rc or
// null), on a carved context-free workspace: kernels only (no memset or
// copy nodes), so that the sequence can be recorded into a HIP graph.
hipError_t accel_run(const MassiveWs& w, const StepConsts& c, const double* m, const double* x,
                     const double* rc, double* acc, hipStream_t s);
// Parameters of the context-free acceleration (one candidate slot, one
// encounter slot: the pair kernel keeps no lists in this form).
genga_params accel_params(const genga_params& p);
// The pair kernel's acceleration mode on the library's own device scratch
// (no workspace argument, no allocation); n <= kAccelNoAllocMax.
constexpr int kAccelNoAllocMax = GENGA_ACCEL_NOALLOC_MAX;
hipError_t accel_noalloc_run(const StepConsts& c, int n, const double* m, const double* x,
                             const double* rc, double* acc, hipStream_t s);

// ---- test-particle mode (tp.hip) --------------------------------------------
size_t tp_carve(TpWs& t, int64_t ntp, int nm, void* base);
// The last step's particle-planet encounters (particle, planet, d2, rc2),
// unsorted (synchronising).
struct TpEnc {
  long long tp;
  int planet;
  double d2, rc2;
};
hipError_t tp_read_encounters(const TpWs& t, std::vector<TpEnc>* out, hipStream_t s);
hipError_t tp_pack(const MassiveWs& w, const TpWs& t, const StepConsts& c,
                   const double* x, const double* v, int coords_in, hipStream_t s);
hipError_t tp_unpack(const MassiveWs& w, const TpWs& t, const StepConsts& c,
                     double* x, double* v, int coords_out, hipStream_t s);
hipError_t tp_prime(const MassiveWs& w, const TpWs& t, const StepConsts& c,
                    hipStream_t s);
hipError_t tp_step(const MassiveWs& w, const TpWs& t, const StepConsts& c,
                   hipStream_t s);
// Sums the per-block counters (synchronising).
hipError_t tp_read_counters(const TpWs& t, TpCounters* h, hipStream_t s);
// Test-particle rows [nm, nm + ntp) of x and v: finite, or all NaN (removed);
// anything else sets *dbad.
hipError_t tp_validate(const TpWs& t, int nm, const double* x, const double* v, int* dbad,
                       hipStream_t s);
// Copies nm + ntp radii (planets first) into the workspace; negative or
// non-finite values set *dbad.
hipError_t tp_set_radii(const TpWs& t, int nm, const double* r, int* dbad, hipStream_t s);

// ---- batched independent systems (batch.hip) --------------------------------
struct BatchSysStat {
  long long steps;               // steps completed since init
  unsigned long long sub;        // accepted BS substeps since init
  unsigned long long enc_total;  // encounters since init
  int nenc;                      // encounters of the last step
  int ngroups;                   // groups of the last step
  int maxg;                      // largest group of the last step
  int kit;                       // largest Kepler iteration count
  unsigned flags;                // latched error bits of this system
  int nlive;                     // bodies left (mergers and ejections remove)
  unsigned long long khist[kKepBins];  // Kepler iterations since init
  double U;                      // internal energy of the system's mergers
};

struct BatchWs {
  int nsys;
  int64_t nb;                      // bodies of all systems
  double4* xm;                     // [nb] x, y, z, m
  double4* vv;                     // [nb] v
  unsigned long long* cand;        // [nb] candidate partners (bits of local indices)
  unsigned long long* encm;        // [nb] encounters j > i of the last step
  double4 *xm2, *vv2;              // copies the tuner runs on
  unsigned long long *cand2, *encm2;
  int* off;                        // [nsys + 1]
  double* m0;                      // [nsys]
  int* order_nat;                  // systems in index order
  int* order_desc;                 // systems by decreasing size
  BatchSysStat* ss;                // [nsys]
  BatchSysStat* ss2;
  int* rslot;                      // [nsys] tableau slice of systems over 8 bodies
  double* rbuf;                    // [nbig] tableaux of the sequential BS
  double* rad;                     // [nb] physical radii (0: no collisions)
  double4* sp;                     // [nb] spins (x, y, z, 0)
  int* ids;                        // [nb] original row of each body
  double4* sp2;                    // the tuner's copies
  int* ids2;
  double* rad2;
  genga_event* ev;                 // [nb] mergers and ejections since init
  unsigned long long* ev_cnt;      // their count (also those beyond nb)
  int coll;                        // some radius is positive
  double rcut, rcut_sun;
  int nmin;
  int nbig;
  int maxn;                        // largest system
  unsigned* flags2;
  int* flag_in;
  DevStat* st;
};

constexpr int kBatchMaxBodies = 64;  // one lane per body
// register budget {1, 2, 4 waves/SIMD} x order (one system per wave), then
// register budget x two systems per wave (systems of up to 32 bodies)
constexpr int kBatchVariants = 9;
constexpr int kBatchPackedVariant0 = 6;

// nbig: systems with more than 8 bodies (each gets a sequential-BS tableau)
size_t batch_carve(BatchWs& b, int nsys, int64_t nb, int nbig, void* base);
hipError_t batch_pack(const BatchWs& b, const double* m, const double* x, const double* v,
                      int coords_in, bool keep_mass, hipStream_t s);
hipError_t batch_unpack(const BatchWs& b, double* x, double* v, int coords_out, hipStream_t s);
hipError_t batch_prime(const BatchWs& b, const StepConsts& c, hipStream_t s);
hipError_t batch_energy(const BatchWs& b, const StepConsts& c, double* E, double* L,
                        hipStream_t s);
// nsteps steps of every system in one launch of the given variant, on the
// live state or on the tuner's copies.
hipError_t batch_run(const BatchWs& b, const StepConsts& c, int variant, int nsteps,
                     bool scratch, hipStream_t s);
hipError_t batch_copy_to_scratch(const BatchWs& b, hipStream_t s);
// Bodies of every system present, original rows, zero spins and radii, no
// events (init).
hipError_t batch_reset_bodies(const BatchWs& b, hipStream_t s);
// Masses of every row replaced (state kept).
hipError_t batch_set_masses(const BatchWs& b, const double* m, hipStream_t s);
const char* batch_variant_name(int v);
// whether variant v can run these systems (two per wave needs sizes <= 32)
bool batch_variant_ok(const BatchWs& b, int v);

// ---- adjoint of the encounter-free map (adj.hip) ----------------------------
// Systems are packed sb lanes each (sb: power of two >= the largest system).
// hybrid adjoint (hadj.hip): checkpoints of T steps every K, and the backward
// pass's workspace (tape of a segment, BS substep starts, Gragg positions)
size_t hadj_ckpt_bytes(int64_t nb, int T, int K);
size_t hadj_work_bytes(int nsys, int K);
hipError_t hadj_forward(const BatchWs& b, const StepConsts& c, int T, int K, double* ckpt,
                        hipStream_t s);
hipError_t hadj_backward(const BatchWs& b, const StepConsts& c, int T, int K, double* ckpt,
                         double* work, const double* gxT, const double* gvT, double* gx0,
                         double* gv0, double* gm, hipStream_t s);

int adj_segment_lanes(int max_n);
size_t adj_tape_bytes(int nsys, int sb, int K);
// T steps of the encounter-free map on the batched state, keeping the state
// every K steps in ckpt ([ceil(T/K)][6][nb]).
hipError_t adj_forward(const BatchWs& b, const StepConsts& c, int sb, int T, int K, double* ckpt,
                       hipStream_t s);
// Gradients of the state before those T steps from the adjoints of the
// state after them (rows x 3), using the checkpoints and a tape.
hipError_t adj_backward(const BatchWs& b, const StepConsts& c, int sb, int T, int K,
                        double* ckpt, double* tape, const double* gxT, const double* gvT,
                        double* gx0, double* gv0, double* gm, hipStream_t s);

// ---- single-operation kernels for component checks (ops.hip) ---------------
hipError_t op_kepler(double mu, int64_t n, const double* x0, const double* v0,
                     double dt, double* x, double* v, int max_iter, int* iters,
                     hipStream_t s);
hipError_t op_hermite(int64_t n, double dt, const double* q, double* out,
                      hipStream_t s);

}  // namespace genga
