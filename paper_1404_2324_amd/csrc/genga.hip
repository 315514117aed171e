// C ABI of the library (include/genga.h): context, workspace validation,
// HIP-graph capture of the step, status reporting.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "genga_impl.h"

using namespace genga;

namespace {

constexpr int kGraphSteps = 16;  // steps per captured graph (and at most 15 in a remainder graph)

int status_from_flags(unsigned f) {
  if (f & F_KEPLER) return GENGA_EKEPLER;
  if (f & F_BS) return GENGA_EBS;
  if (f & (F_CAND_OVF | F_ENC_OVF | F_TP_OVF | F_ADJ_LEAF)) return GENGA_EOVERFLOW;
  if (f & F_GROUP) return GENGA_EGROUP;
  if (f & F_ADJ_ENC) return GENGA_EADJ_ENCOUNTER;
  if (f & F_NMIN) return GENGA_WNMIN;
  if (f & F_SYS_STOP) return GENGA_WSTOPPED;
  return GENGA_OK;
}

}  // namespace

bool genga::params_valid(const genga_params* p) {
  if (!p) return false;
  const double v[] = {p->G, p->m0, p->dt, p->n1, p->n2, p->pf, p->bs_tol, p->rcut, p->rcut_sun};
  for (double d : v)
    if (!std::isfinite(d)) return false;
  double w[8];
  return p->G > 0.0 && p->m0 > 0.0 && p->dt != 0.0 && p->n1 >= 0.0 && p->n2 >= 0.0 &&
         p->pf >= 1.0 && p->bs_max_depth >= 0 && p->bs_max_depth <= 40 &&
         p->kepler_max_iter >= 1 && p->cand_per_body >= 1 && p->enc_cap >= 1 &&
         composition(p->order, w) > 0 && p->rcut >= 0.0 && p->rcut_sun >= 0.0 && p->nmin >= 0;
}

namespace {

bool params_ok(const genga_params* p) { return params_valid(p); }

int max_bodies(const genga_params* p) { return p->encounter_free ? 65536 : kGroupMaxN; }

constexpr int64_t kTpMaxParticles = 1ll << 30;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int kBatchMaxSystems = 1 << 24;

bool shape_ok(int mode, const genga_params* p, int nm, int64_t ntp, int nsys = 0,
              int64_t nbod = 0) {
  if (p->order > 2 && mode != GENGA_MASSIVE) return false;  // compositions: main mode
  // bodies leaving (rcut, rcut_sun, nmin): main mode at second order with
  // encounters, and batched mode
  const bool leave = p->rcut > 0.0 || p->rcut_sun > 0.0 || p->nmin > 0;
  if (leave && mode == GENGA_TEST) return false;
  if (leave && mode == GENGA_MASSIVE && (p->order > 2 || p->encounter_free)) return false;
  if (mode == GENGA_MASSIVE) return nm >= 1 && nm <= max_bodies(p) && ntp == 0;
  if (mode == GENGA_TEST) return nm >= 1 && nm <= kTpMaxPlanets && ntp >= 0 && ntp <= kTpMaxParticles;
  if (mode == GENGA_BATCH)
    return nsys >= 1 && nsys <= kBatchMaxSystems && nbod >= nsys &&
           nbod <= (int64_t)nsys * kBatchMaxBodies;
  return false;
}

size_t ws_bytes(int mode, const genga_params& p, int nm, int64_t ntp, int nsys = 0,
                int64_t nbod = 0) {
  if (mode == GENGA_TEST) {
    TpWs t;
    return align256(massive_ws_bytes(nm, p, true)) + tp_carve(t, ntp, nm, nullptr);
  }
  if (mode == GENGA_BATCH) {
    BatchWs b;
    return batch_carve(b, nsys, nbod, nsys, nullptr);
  }
  return massive_ws_bytes(nm, p, false);
}

constexpr int kTuneSteps = 4;

}  // namespace

struct genga_ctx {
  int mode = GENGA_MASSIVE;
  genga_params p{};
  StepConsts c{};
  MassiveWs w{};
  TpWs t{};
  BatchWs b{};
  int variant = 0;                       // batched: the tuner's choice
  double tune_us[kBatchVariants] = {};   // batched: the tuner's timings
  hipGraphExec_t g_batch = nullptr;      // batched: one launch of g_batch_steps steps
  int g_batch_steps = 0;
  int sb = 64;                           // batched: lanes per system in the adjoint
  double* adj_ckpt = nullptr;            // the last genga_adj_forward's buffer
  size_t adj_bytes = 0;
  int adj_T = 0, adj_K = 0;
  std::vector<StepConsts> sub;           // main mode: the constants of each sub-step
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t g_many = nullptr;
  hipGraphExec_t g_rem[16] = {};  // r steps in one graph, r = 1 .. 15
  int64_t steps = 0;
  bool tuned = false;                    // batched mode: the tuner has chosen a variant
};

#define HIPCHK(expr)                          \
  do {                                        \
    if ((expr) != hipSuccess) return GENGA_EHIP; \
  } while (0)

// Captured step graphs are dropped when the step's launches change.
static void drop_graphs(genga_ctx* ctx) {
  if (ctx->g_many) (void)hipGraphExecDestroy(ctx->g_many);
  ctx->g_many = nullptr;
  for (hipGraphExec_t& g : ctx->g_rem) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

static int capture(genga_ctx* ctx, int nsteps, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
    for (size_t q = 0; q < ctx->sub.size() && e == hipSuccess; ++q)
      e = massive_step(ctx->w, ctx->sub[q], ctx->cap);
    if (e == hipSuccess && ctx->mode == GENGA_TEST) e = tp_step(ctx->w, ctx->t, ctx->c, ctx->cap);
  }
  hipError_t e2 = hipStreamEndCapture(ctx->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return GENGA_EHIP;
  }
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e == hipSuccess ? GENGA_OK : GENGA_EHIP;
}

static int read_status(genga_ctx* ctx, DevStat* hs) {
  HIPCHK(hipMemcpyAsync(hs, ctx->w.st, sizeof(DevStat), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return GENGA_OK;
}

static int load_state(genga_ctx* ctx, const double* d_m, const double* d_x, const double* d_v,
                      int coords_in) {
  const int n = ctx->w.n;
  const int64_t rows = n + (ctx->mode == GENGA_TEST ? ctx->t.ntp : 0);
  HIPCHK(hipMemsetAsync(ctx->w.flag_in, 0, sizeof(int), ctx->stream));
  if (d_m) HIPCHK(validate_finite(d_m, n, ctx->w.flag_in, ctx->stream));
  // massive rows finite; test-particle rows finite or all NaN (removed)
  HIPCHK(validate_finite(d_x, 3 * (int64_t)n, ctx->w.flag_in, ctx->stream));
  HIPCHK(validate_finite(d_v, 3 * (int64_t)n, ctx->w.flag_in, ctx->stream));
  if (ctx->mode == GENGA_TEST)
    HIPCHK(tp_validate(ctx->t, n, d_x, d_v, ctx->w.flag_in, ctx->stream));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, ctx->w.flag_in, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (bad) return GENGA_EINVAL;
  HIPCHK(massive_pack(ctx->w, ctx->c, d_m, d_x, d_v, coords_in, ctx->stream));
  if (ctx->mode == GENGA_TEST) HIPCHK(tp_pack(ctx->w, ctx->t, ctx->c, d_x, d_v, coords_in, ctx->stream));
  HIPCHK(massive_prime(ctx->w, ctx->sub[0], ctx->stream));
  if (ctx->mode == GENGA_TEST) HIPCHK(tp_prime(ctx->w, ctx->t, ctx->c, ctx->stream));
  return GENGA_OK;
}

// The constants of each sub-step of the (composed) step: dt_k = w_k dt, the
// radii formed at its end with the next sub-step's |dt|, and (orders above
// two) the encounter search over all pairs.
static void make_substeps(genga_ctx* ctx) {
  double w[8];
  const int K = composition(ctx->p.order, w);
  ctx->sub.clear();
  for (int k = 0; k < K; ++k) {
    genga_params q = ctx->p;
    q.dt = w[k] * ctx->p.dt;
    StepConsts c = make_consts(q);
    c.absdt_next = fabs(w[(k + 1) % K] * ctx->p.dt);
    c.all_pairs = K > 1;
    ctx->sub.push_back(c);
  }
}

// ---- batched mode -----------------------------------------------------------
static int batch_capture(genga_ctx* ctx, int nsteps) {
  if (ctx->g_batch) {
    (void)hipGraphExecDestroy(ctx->g_batch);
    ctx->g_batch = nullptr;
  }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
  const hipError_t e = batch_run(ctx->b, ctx->c, ctx->variant, nsteps, false, ctx->cap);
  const hipError_t e2 = hipStreamEndCapture(ctx->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return GENGA_EHIP;
  }
  const hipError_t e3 = hipGraphInstantiate(&ctx->g_batch, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) return GENGA_EHIP;
  ctx->g_batch_steps = nsteps;
  return GENGA_OK;
}

// Runs every variant for `steps` steps on a copy of the current state and
// keeps the fastest for later steps.
static int batch_tune(genga_ctx* ctx, int steps) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return GENGA_EHIP;
  }
  int rc = GENGA_OK, best = -1;
  for (int v = 0; v < kBatchVariants && rc == GENGA_OK; ++v) {
    ctx->tune_us[v] = -1.0;  // variants that cannot run these systems
    if (!batch_variant_ok(ctx->b, v)) continue;
    float ms = 0.0f;
    if (batch_copy_to_scratch(ctx->b, ctx->stream) != hipSuccess ||
        hipEventRecord(e0, ctx->stream) != hipSuccess ||
        batch_run(ctx->b, ctx->c, v, steps, true, ctx->stream) != hipSuccess ||
        hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      rc = GENGA_EHIP;
    ctx->tune_us[v] = ms * 1e3;
    if (best < 0 || ctx->tune_us[v] < ctx->tune_us[best]) best = v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != GENGA_OK) return rc;
  ctx->tuned = true;
  if (best != ctx->variant || !ctx->g_batch) {
    ctx->variant = best;
    if (ctx->g_batch) {
      (void)hipGraphExecDestroy(ctx->g_batch);
      ctx->g_batch = nullptr;
    }
  }
  return GENGA_OK;
}

static int batch_load(genga_ctx* ctx, const double* d_m, const double* d_x, const double* d_v,
                      int coords_in) {
  const BatchWs& b = ctx->b;
  HIPCHK(hipMemsetAsync(b.flag_in, 0, sizeof(int), ctx->stream));
  if (d_m) HIPCHK(validate_finite(d_m, b.nb, b.flag_in, ctx->stream));
  HIPCHK(validate_finite(d_x, 3 * b.nb, b.flag_in, ctx->stream));
  HIPCHK(validate_finite(d_v, 3 * b.nb, b.flag_in, ctx->stream));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, b.flag_in, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (bad) return GENGA_EINVAL;
  HIPCHK(batch_pack(b, d_m, d_x, d_v, coords_in, d_m == nullptr, ctx->stream));
  HIPCHK(batch_prime(b, ctx->c, ctx->stream));
  return GENGA_OK;
}

static int batch_init(genga_ctx** out, const genga_params* p, int n_sys,
                      const int32_t* d_offsets, const double* d_m0, const double* d_m,
                      const double* d_x, const double* d_v, int coords_in, void* d_workspace,
                      size_t ws_bytes_in, void* stream) {
  if (!params_ok(p) || n_sys < 1 || n_sys > kBatchMaxSystems || !d_offsets) return GENGA_EINVAL;
  if (!d_m || !d_x || !d_v || !d_workspace) return GENGA_EINVAL;
  if (coords_in != GENGA_HELIO && coords_in != GENGA_DEMOCRATIC) return GENGA_EINVAL;
  if (((uintptr_t)d_workspace & 255u) != 0) return GENGA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  // the system layout is read once on the host: sizes 1..64, contiguous
  std::vector<int32_t> off((size_t)n_sys + 1);
  HIPCHK(hipMemcpyAsync(off.data(), d_offsets, off.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost, st));
  std::vector<double> m0((size_t)n_sys, p->m0);
  if (d_m0)
    HIPCHK(hipMemcpyAsync(m0.data(), d_m0, m0.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (off[0] != 0) return GENGA_EINVAL;
  int nbig = 0;
  for (int s = 0; s < n_sys; ++s) {
    const int n = off[s + 1] - off[s];
    if (n < 1 || n > kBatchMaxBodies) return GENGA_EINVAL;
    if (!(m0[s] > 0.0) || !std::isfinite(m0[s])) return GENGA_EINVAL;
    if (n > 8) ++nbig;
  }
  const int64_t nb = off[n_sys];
  if (!shape_ok(GENGA_BATCH, p, 0, 0, n_sys, nb)) return GENGA_EINVAL;
  if (ws_bytes_in < ws_bytes(GENGA_BATCH, *p, 0, 0, n_sys, nb)) return GENGA_ENOMEM;
  genga_ctx* ctx = new (std::nothrow) genga_ctx();
  if (!ctx) return GENGA_ENOMEM;
  ctx->mode = GENGA_BATCH;
  ctx->p = *p;
  ctx->c = make_consts(*p);
  ctx->stream = st;
  batch_carve(ctx->b, n_sys, nb, n_sys, d_workspace);
  ctx->b.coll = 0;
  ctx->b.rcut = p->rcut;
  ctx->b.rcut_sun = p->rcut_sun;
  ctx->b.nmin = p->nmin;
  ctx->w.st = ctx->b.st;  // the status word read by the common calls
  std::vector<int> order(n_sys), desc(n_sys), rslot(n_sys, 0);
  for (int s = 0; s < n_sys; ++s) order[s] = s;
  desc = order;
  std::stable_sort(desc.begin(), desc.end(), [&](int a, int b) {
    return off[a + 1] - off[a] > off[b + 1] - off[b];
  });
  int maxn = 1;
  for (int s = 0, k = 0; s < n_sys; ++s) {
    if (off[s + 1] - off[s] > 8) rslot[s] = k++;
    maxn = std::max(maxn, off[s + 1] - off[s]);
  }
  ctx->sb = adj_segment_lanes(maxn);
  ctx->b.maxn = maxn;
  (void)nbig;
  int rc = GENGA_OK;
  if (hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) rc = GENGA_EHIP;
  const BatchWs& b = ctx->b;
  if (rc == GENGA_OK &&
      (hipMemcpyAsync(b.off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(b.m0, m0.data(), m0.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(b.order_nat, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(b.order_desc, desc.data(), desc.size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(b.rslot, rslot.data(), rslot.size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemsetAsync(b.ss, 0, (size_t)n_sys * sizeof(BatchSysStat), st) != hipSuccess ||
       hipMemsetAsync(b.st, 0, sizeof(DevStat), st) != hipSuccess ||
       batch_reset_bodies(b, st) != hipSuccess))
    rc = GENGA_EHIP;
  if (rc == GENGA_OK) rc = batch_load(ctx, d_m, d_x, d_v, coords_in);
  if (rc == GENGA_OK && hipStreamSynchronize(st) != hipSuccess) rc = GENGA_EHIP;
  if (rc != GENGA_OK) {
    genga_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return GENGA_OK;
}

static int batch_step(genga_ctx* ctx, int64_t nsteps) {
  // the tuner runs before the first steps (not at init: contexts that only
  // take the adjoint never launch the step kernel)
  if (!ctx->tuned) {
    const int r = batch_tune(ctx, kTuneSteps);
    if (r != GENGA_OK) return r;
  }
  while (nsteps > 0) {
    const int chunk = (int)std::min<int64_t>(nsteps, 1 << 30);
    if (!ctx->g_batch || ctx->g_batch_steps != chunk) {
      const int r = batch_capture(ctx, chunk);
      if (r != GENGA_OK) return r;
    }
    HIPCHK(hipGraphLaunch(ctx->g_batch, ctx->stream));
    ctx->steps += chunk;
    nsteps -= chunk;
  }
  return GENGA_OK;
}

extern "C" {

void genga_params_default(genga_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->G = 1.0;
  p->m0 = 1.0;
  p->dt = 0.02 * M_PI;
  p->n1 = 3.0;
  p->n2 = 0.4;
  p->pf = 3.0;
  p->bs_tol = 1e-13;
  p->bs_max_depth = 20;
  p->kepler_max_iter = 40;
  p->encounter_free = 0;
  p->cand_per_body = 32;
  p->enc_cap = 16384;
}

size_t genga_workspace_bytes(int mode, const genga_params* p, int n_massive, int64_t n_test,
                             int n_sys, int64_t n_bodies) {
  if (!params_ok(p) || !shape_ok(mode, p, n_massive, n_test, n_sys, n_bodies)) return 0;
  return ws_bytes(mode, *p, n_massive, n_test, n_sys, n_bodies);
}

int genga_init(genga_ctx** out, int mode, const genga_params* p, int n_massive, int64_t n_test,
               int n_sys, const int32_t* d_offsets, const double* d_m0, const double* d_m,
               const double* d_x, const double* d_v, int coords_in, void* d_workspace,
               size_t ws_bytes_in, void* stream) {
  if (!out) return GENGA_EINVAL;
  *out = nullptr;
  if (mode == GENGA_BATCH)
    return batch_init(out, p, n_sys, d_offsets, d_m0, d_m, d_x, d_v, coords_in, d_workspace,
                      ws_bytes_in, stream);
  if (!params_ok(p) || !shape_ok(mode, p, n_massive, n_test)) return GENGA_EINVAL;
  if (!d_m || !d_x || !d_v || !d_workspace) return GENGA_EINVAL;
  if (coords_in != GENGA_HELIO && coords_in != GENGA_DEMOCRATIC) return GENGA_EINVAL;
  if (((uintptr_t)d_workspace & 255u) != 0) return GENGA_EINVAL;
  const size_t need = ws_bytes(mode, *p, n_massive, n_test);
  if (ws_bytes_in < need) return GENGA_ENOMEM;
  genga_ctx* ctx = new (std::nothrow) genga_ctx();
  if (!ctx) return GENGA_ENOMEM;
  ctx->mode = mode;
  ctx->p = *p;
  ctx->c = make_consts(*p);
  make_substeps(ctx);
  ctx->stream = (hipStream_t)stream;
  const bool tp = mode == GENGA_TEST;
  const size_t moff = align256(massive_carve(ctx->w, n_massive, *p, d_workspace, tp));
  if (tp) tp_carve(ctx->t, n_test, n_massive, (char*)d_workspace + moff);
  int rc = GENGA_OK;
  if (hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) rc = GENGA_EHIP;
  if (rc == GENGA_OK &&
      (hipMemsetAsync(ctx->w.st, 0, sizeof(DevStat), ctx->stream) != hipSuccess ||
       hipMemsetAsync(ctx->w.khist, 0, (size_t)ctx->w.nblk * kKepBins * sizeof(unsigned long long),
                      ctx->stream) != hipSuccess ||
       massive_reset_bodies(ctx->w, true, ctx->stream) != hipSuccess))
    rc = GENGA_EHIP;
  if (rc == GENGA_OK && tp &&
      (hipMemsetAsync(ctx->t.rad, 0, (kTpMaxPlanets + std::max<int64_t>(n_test, 1)) * sizeof(double),
                      ctx->stream) != hipSuccess ||
       hipMemsetAsync(ctx->t.cum, 0, ctx->t.cum_bytes, ctx->stream) != hipSuccess))
    rc = GENGA_EHIP;
  if (rc == GENGA_OK) rc = load_state(ctx, d_m, d_x, d_v, coords_in);
  if (rc == GENGA_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = GENGA_EHIP;
  if (rc != GENGA_OK) {
    genga_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return GENGA_OK;
}

int genga_step(genga_ctx* ctx, int64_t nsteps) {
  if (!ctx || nsteps < 0) return GENGA_EINVAL;
  if (nsteps == 0) return GENGA_OK;
  if (ctx->mode == GENGA_BATCH) return batch_step(ctx, nsteps);
  if (nsteps >= kGraphSteps && !ctx->g_many) {
    int r = capture(ctx, kGraphSteps, &ctx->g_many);
    if (r != GENGA_OK) return r;
  }
  // the remaining steps as one graph of their own, so that a call's time per
  // step does not depend on how its count divides into graphs of 16
  const int rem = (int)(nsteps % kGraphSteps);
  if (rem && !ctx->g_rem[rem]) {
    int r = capture(ctx, rem, &ctx->g_rem[rem]);
    if (r != GENGA_OK) return r;
  }
  for (int64_t k = 0; k < nsteps / kGraphSteps; ++k) HIPCHK(hipGraphLaunch(ctx->g_many, ctx->stream));
  if (rem) HIPCHK(hipGraphLaunch(ctx->g_rem[rem], ctx->stream));
  ctx->steps += nsteps;
  return GENGA_OK;
}

// Steps with event pairs around kernel slots (all of them, or only the pair
// kernel's); us[k] is slot k's average dispatch duration in microseconds
// (0 for slots the mode does not launch).  One event pair per slot and step,
// read after the last step: the steps run back to back as in a graph replay.
static_assert(GENGA_STEP_KERNELS == kStepKernels, "kernels per step");
static int step_timed(genga_ctx* ctx, int64_t nsteps, bool all, double* us) {
  constexpr int K = kStepKernels;
  std::vector<hipEvent_t> ev((size_t)(2 * K * nsteps), nullptr);
  const bool enc = !ctx->c.encounter_free;
  // the pair kernel always; with all, every kernel the step launches
  auto timed = [&](int k) {
    return k == kSlotPairs || (all && (enc || k == 0 || k == K - 1));
  };
  const int klast = all ? K - 1 : kSlotPairs;  // the last timed slot of a step
  int rc = GENGA_OK;
  for (int64_t t = 0; t < nsteps && rc == GENGA_OK; ++t)
    for (int k = 0; k < K && rc == GENGA_OK; ++k)
      if (timed(k))
        for (int q = 0; q < 2; ++q)
          if (hipEventCreate(&ev[(size_t)(2 * (K * t + k) + q)]) != hipSuccess) rc = GENGA_EHIP;
  hipEvent_t last = nullptr;
  for (int64_t t = 0; t < nsteps && rc == GENGA_OK; ++t) {
    const hipEvent_t* kev = &ev[(size_t)(2 * K * t)];
    if (massive_step(ctx->w, ctx->sub[0], ctx->stream, kev) != hipSuccess ||
        (ctx->mode == GENGA_TEST && tp_step(ctx->w, ctx->t, ctx->c, ctx->stream) != hipSuccess))
      rc = GENGA_EHIP;
    last = kev[2 * klast + 1];
  }
  if (rc == GENGA_OK && hipEventSynchronize(last) != hipSuccess) rc = GENGA_EHIP;
  for (int k = 0; k < K; ++k) us[k] = 0.0;
  for (int64_t t = 0; t < nsteps && rc == GENGA_OK; ++t)
    for (int k = 0; k < K && rc == GENGA_OK; ++k) {
      if (!timed(k)) continue;
      float ms = 0.0f;
      const size_t i = (size_t)(2 * (K * t + k));
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) rc = GENGA_EHIP;
      us[k] += ms * 1e3 / (double)nsteps;
    }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rc != GENGA_OK) return rc;
  ctx->steps += nsteps;
  return genga_sync(ctx);
}

int genga_step_profiled(genga_ctx* ctx, int64_t nsteps, double* h_kick_us) {
  if (!ctx || nsteps < 1 || nsteps > 4096 || !h_kick_us || ctx->mode == GENGA_BATCH ||
      ctx->sub.size() != 1)
    return GENGA_EINVAL;
  double us[kStepKernels];
  const int r = step_timed(ctx, nsteps, false, us);
  if (r >= 0) *h_kick_us = us[kSlotPairs];
  return r;
}

int genga_step_kernel_us(genga_ctx* ctx, int64_t nsteps, double* h_us) {
  if (!ctx || nsteps < 1 || nsteps > 512 || !h_us || ctx->mode == GENGA_BATCH ||
      ctx->sub.size() != 1)
    return GENGA_EINVAL;
  return step_timed(ctx, nsteps, true, h_us);
}

int genga_sync(genga_ctx* ctx) {
  if (!ctx) return GENGA_EINVAL;
  DevStat hs;
  int r = read_status(ctx, &hs);
  if (r != GENGA_OK) return r;
  return status_from_flags(hs.flags);
}

int genga_get_state(genga_ctx* ctx, double* d_x, double* d_v, int coords_out) {
  if (!ctx || !d_x || !d_v) return GENGA_EINVAL;
  if (coords_out != GENGA_HELIO && coords_out != GENGA_DEMOCRATIC) return GENGA_EINVAL;
  if (ctx->mode == GENGA_BATCH) {
    HIPCHK(batch_unpack(ctx->b, d_x, d_v, coords_out, ctx->stream));
    return genga_sync(ctx);
  }
  HIPCHK(massive_unpack(ctx->w, ctx->c, d_x, d_v, coords_out, ctx->stream));
  if (ctx->mode == GENGA_TEST) HIPCHK(tp_unpack(ctx->w, ctx->t, ctx->c, d_x, d_v, coords_out, ctx->stream));
  return genga_sync(ctx);
}

int genga_set_state(genga_ctx* ctx, const double* d_x, const double* d_v, int coords_in) {
  if (!ctx || !d_x || !d_v) return GENGA_EINVAL;
  if (coords_in != GENGA_HELIO && coords_in != GENGA_DEMOCRATIC) return GENGA_EINVAL;
  if (ctx->mode == GENGA_BATCH) {
    const int r = batch_load(ctx, nullptr, d_x, d_v, coords_in);
    if (r != GENGA_OK) return r;
    return genga_sync(ctx);
  }
  // masses stay: the pre-drift scratch holds them while the state is repacked
  double* dm = reinterpret_cast<double*>(ctx->w.xpre);
  HIPCHK(massive_masses(ctx->w, dm, ctx->stream));
  int r = load_state(ctx, dm, d_x, d_v, coords_in);
  if (r != GENGA_OK) return r;
  return genga_sync(ctx);
}

int genga_set_masses(genga_ctx* ctx, const double* d_m) {
  if (!ctx || !d_m || ctx->mode != GENGA_BATCH) return GENGA_EINVAL;
  const BatchWs& b = ctx->b;
  HIPCHK(hipMemsetAsync(b.flag_in, 0, sizeof(int), ctx->stream));
  HIPCHK(validate_finite(d_m, b.nb, b.flag_in, ctx->stream));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, b.flag_in, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (bad) return GENGA_EINVAL;
  HIPCHK(batch_set_masses(b, d_m, ctx->stream));
  HIPCHK(batch_prime(b, ctx->c, ctx->stream));
  return genga_sync(ctx);
}

int genga_energy(genga_ctx* ctx, double* d_E, double* d_L) {
  if (!ctx || !d_E || !d_L) return GENGA_EINVAL;
  if (ctx->mode == GENGA_BATCH) {
    HIPCHK(batch_energy(ctx->b, ctx->c, d_E, d_L, ctx->stream));
    return GENGA_OK;
  }
  HIPCHK(massive_energy(ctx->w, ctx->c, d_E, d_L, ctx->stream));
  return GENGA_OK;
}

int genga_accel_state(genga_ctx* ctx, double* d_acc) {
  if (!ctx || !d_acc || ctx->mode == GENGA_BATCH) return GENGA_EINVAL;
  HIPCHK(massive_accel(ctx->w, ctx->c, ctx->w.xs, d_acc, ctx->stream));
  return GENGA_OK;
}

// Pairs i < j (global rows) of per-body partner masks of the batched layout.
static int batch_pairs(genga_ctx* ctx, const unsigned long long* d_mask,
                       std::vector<std::pair<int, int>>* pairs) {
  const BatchWs& b = ctx->b;
  std::vector<unsigned long long> mk((size_t)b.nb);
  std::vector<int32_t> off((size_t)b.nsys + 1);
  HIPCHK(hipMemcpyAsync(mk.data(), d_mask, mk.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipMemcpyAsync(off.data(), b.off, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int s = 0; s < b.nsys; ++s)
    for (int i = off[s]; i < off[s + 1]; ++i)
      for (int j = i + 1; j < off[s + 1]; ++j)
        if ((mk[i] >> (j - off[s])) & 1ull) pairs->emplace_back(i, j);
  return GENGA_OK;
}

int genga_encounters(genga_ctx* ctx, int32_t* h_ij, double* h_dmin2, double* h_rc2, int cap,
                     int* h_n) {
  if (!ctx || !h_n || cap < 0 || (cap > 0 && !h_ij)) return GENGA_EINVAL;
  DevStat hs;
  int r = read_status(ctx, &hs);
  if (r != GENGA_OK) return r;
  if (ctx->mode == GENGA_BATCH) {
    std::vector<std::pair<int, int>> pr;
    if (ctx->steps > 0) {
      r = batch_pairs(ctx, ctx->b.encm, &pr);
      if (r != GENGA_OK) return r;
    }
    const int np = (int)pr.size();
    for (int k = 0; k < std::min(np, cap); ++k) {
      h_ij[2 * k] = pr[k].first;
      h_ij[2 * k + 1] = pr[k].second;
      if (h_dmin2) h_dmin2[k] = std::nan("");
      if (h_rc2) h_rc2[k] = std::nan("");
    }
    *h_n = np;
    if (np > cap) return GENGA_EOVERFLOW;
    return status_from_flags(hs.flags);
  }
  const int n = ctx->p.encounter_free || ctx->steps == 0 ? 0 : hs.nenc;
  const int have = std::min(n, ctx->w.enc_cap);
  std::vector<int2> ij(have);
  std::vector<double> d2(have), rc2(have);
  if (have > 0) {
    HIPCHK(hipMemcpyAsync(ij.data(), ctx->w.encij, have * sizeof(int2), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(d2.data(), ctx->w.encd2, have * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(rc2.data(), ctx->w.encrc2, have * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  std::vector<int> idx(have);
  for (int k = 0; k < have; ++k) idx[k] = k;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) {
    return ij[a].x != ij[b].x ? ij[a].x < ij[b].x : ij[a].y < ij[b].y;
  });
  const int wr = std::min(have, cap);
  for (int k = 0; k < wr; ++k) {
    h_ij[2 * k] = ij[idx[k]].x;
    h_ij[2 * k + 1] = ij[idx[k]].y;
    if (h_dmin2) h_dmin2[k] = d2[idx[k]];
    if (h_rc2) h_rc2[k] = rc2[idx[k]];
  }
  *h_n = n;
  if (n > cap || n > ctx->w.enc_cap) return GENGA_EOVERFLOW;
  return status_from_flags(hs.flags);
}

int genga_candidates(genga_ctx* ctx, int32_t* h_ij, double* h_r2, int cap, int* h_n) {
  if (!ctx || !h_n || cap < 0 || (cap > 0 && !h_ij)) return GENGA_EINVAL;
  DevStat hs;
  int r = read_status(ctx, &hs);
  if (r != GENGA_OK) return r;
  if (ctx->mode == GENGA_BATCH) {
    std::vector<std::pair<int, int>> pr;
    r = batch_pairs(ctx, ctx->b.cand, &pr);
    if (r != GENGA_OK) return r;
    const int np = (int)pr.size();
    for (int k = 0; k < std::min(np, cap); ++k) {
      h_ij[2 * k] = pr[k].first;
      h_ij[2 * k + 1] = pr[k].second;
      if (h_r2) h_r2[k] = std::nan("");
    }
    *h_n = np;
    if (np > cap) return GENGA_EOVERFLOW;
    return status_from_flags(hs.flags);
  }
  const int n = ctx->w.n, cpb = ctx->w.cpb;
  std::vector<int> cnt(n), tab((size_t)n * cpb);
  std::vector<double> r2((size_t)n * cpb);
  HIPCHK(hipMemcpyAsync(cnt.data(), ctx->w.ccnt, n * sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipMemcpyAsync(tab.data(), ctx->w.ctab, (size_t)n * cpb * sizeof(int),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipMemcpyAsync(r2.data(), ctx->w.cr2, (size_t)n * cpb * sizeof(double),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  // (i, j, slot of the pair in row i)
  std::vector<std::tuple<int, int, size_t>> pairs;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < std::min(cnt[i], cpb); ++k) {
      const size_t at = (size_t)i * cpb + k;
      if (tab[at] > i) pairs.emplace_back(i, tab[at], at);
    }
  std::sort(pairs.begin(), pairs.end());
  const int np = (int)pairs.size();
  for (int k = 0; k < std::min(np, cap); ++k) {
    h_ij[2 * k] = std::get<0>(pairs[k]);
    h_ij[2 * k + 1] = std::get<1>(pairs[k]);
    if (h_r2) h_r2[k] = r2[std::get<2>(pairs[k])];
  }
  *h_n = np;
  if (np > cap) return GENGA_EOVERFLOW;
  return status_from_flags(hs.flags);
}

int genga_stats(genga_ctx* ctx, genga_stats_t* s) {
  if (!ctx || !s) return GENGA_EINVAL;
  DevStat hs;
  int r = read_status(ctx, &hs);
  if (r != GENGA_OK) return r;
  std::memset(s, 0, sizeof(*s));
  s->steps = ctx->steps;
  if (ctx->mode == GENGA_BATCH) {
    std::vector<BatchSysStat> ss((size_t)ctx->b.nsys);
    HIPCHK(hipMemcpyAsync(ss.data(), ctx->b.ss, ss.size() * sizeof(BatchSysStat),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (const BatchSysStat& t : ss) {
      for (int q = 0; q < kKepBins; ++q) s->kepler_hist[q] += (int64_t)t.khist[q];
      s->n_enc += ctx->steps > 0 ? t.nenc : 0;
      s->n_groups += ctx->steps > 0 ? t.ngroups : 0;
      s->max_group = std::max(s->max_group, t.maxg);
      s->kepler_iter_max = std::max(s->kepler_iter_max, t.kit);
      s->bs_substeps += (int64_t)t.sub;
      s->enc_total += (int64_t)t.enc_total;
    }
    s->flags = hs.flags;
    return status_from_flags(hs.flags);
  }
  const bool any = ctx->steps > 0 && !ctx->p.encounter_free;
  s->n_cand = any ? hs.ncand : 0;
  s->n_enc = any ? hs.nenc : 0;
  s->n_groups = any ? hs.ngroups : 0;
  s->max_group = any ? hs.maxg : 0;
  TpCounters tc = {};
  if (ctx->mode == GENGA_TEST) HIPCHK(tp_read_counters(ctx->t, &tc, ctx->stream));
  std::vector<unsigned long long> kh((size_t)ctx->w.nblk * kKepBins);
  HIPCHK(hipMemcpyAsync(kh.data(), ctx->w.khist, kh.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (size_t q = 0; q < kh.size(); ++q) s->kepler_hist[q % kKepBins] += (int64_t)kh[q];
  for (int q = 0; q < kKepBins; ++q) s->kepler_hist[q] += (int64_t)tc.khist[q];
  s->kepler_iter_max = std::max(hs.kep_itmax, tc.kit);
  s->tp_enc = ctx->steps > 0 && !ctx->p.encounter_free ? (int32_t)tc.enc : 0;
  s->bs_substeps = (int64_t)(hs.bs_sub + tc.sub);
  s->enc_total = (int64_t)hs.enc_total;
  s->full_kicks = (int64_t)hs.fullkicks;
  s->tp_enc_total = (int64_t)tc.enc_total;
  s->tp_removed = (int64_t)hs.tp_removed;
  s->flags = hs.flags;
  return status_from_flags(hs.flags);
}

int genga_tp_encounters(genga_ctx* ctx, int64_t* h_tp, int32_t* h_planet, double* h_d2,
                        double* h_rc2, int64_t cap, int64_t* h_n) {
  if (!ctx || !h_n || cap < 0 || ctx->mode != GENGA_TEST) return GENGA_EINVAL;
  if (cap > 0 && (!h_tp || !h_planet)) return GENGA_EINVAL;
  DevStat hs;
  int r = read_status(ctx, &hs);
  if (r != GENGA_OK) return r;
  std::vector<TpEnc> e;
  if (ctx->steps > 0 && !ctx->p.encounter_free) HIPCHK(tp_read_encounters(ctx->t, &e, ctx->stream));
  std::sort(e.begin(), e.end(), [](const TpEnc& a, const TpEnc& b) {
    return a.tp != b.tp ? a.tp < b.tp : a.planet < b.planet;
  });
  const int64_t n = (int64_t)e.size(), wr = std::min(n, cap);
  for (int64_t k = 0; k < wr; ++k) {
    h_tp[k] = e[k].tp;
    h_planet[k] = e[k].planet;
    if (h_d2) h_d2[k] = e[k].d2;
    if (h_rc2) h_rc2[k] = e[k].rc2;
  }
  *h_n = n;
  if (n > cap) return GENGA_EOVERFLOW;
  return status_from_flags(hs.flags);
}

int genga_set_radii(genga_ctx* ctx, const double* d_radii) {
  if (!ctx || !d_radii) return GENGA_EINVAL;
  if (ctx->mode == GENGA_BATCH) {
    // one radius per row; any positive one turns the mergers on
    const BatchWs& b = ctx->b;
    std::vector<double> r((size_t)b.nb);
    HIPCHK(hipMemcpyAsync(r.data(), d_radii, r.size() * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    bool any = false;
    for (double q : r) {
      if (!(q >= 0.0) || !std::isfinite(q)) return GENGA_EINVAL;
      any = any || q > 0.0;
    }
    HIPCHK(hipMemcpyAsync(b.rad, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if ((int)any != ctx->b.coll && ctx->g_batch) {
      (void)hipGraphExecDestroy(ctx->g_batch);  // the launch changes kernel
      ctx->g_batch = nullptr;
    }
    ctx->b.coll = any ? 1 : 0;
    return GENGA_OK;
  }
  if (ctx->mode == GENGA_MASSIVE) {
    // one radius per row (bodies that left keep theirs); any positive one
    // turns the collision tests on (second order with encounters only)
    if (ctx->sub.size() != 1 || ctx->p.encounter_free) return GENGA_EINVAL;
    const int n = ctx->w.n;
    std::vector<double> r((size_t)n);
    HIPCHK(hipMemcpyAsync(r.data(), d_radii, r.size() * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    bool any = false;
    for (double q : r) {
      if (!(q >= 0.0) || !std::isfinite(q)) return GENGA_EINVAL;
      any = any || q > 0.0;
    }
    HIPCHK(hipMemcpyAsync(ctx->w.rad, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    StepConsts& c = ctx->sub[0];
    const int coll = any ? 1 : 0;
    const int phys = coll || c.rcut > 0.0 || c.rcut_sun > 0.0 || c.nmin > 0;
    if (coll != c.coll || phys != c.phys) {
      c.coll = coll;
      c.phys = phys;
      drop_graphs(ctx);  // the step's launches change
    }
    return GENGA_OK;
  }
  if (ctx->mode != GENGA_TEST) return GENGA_EINVAL;
  HIPCHK(hipMemsetAsync(ctx->w.flag_in, 0, sizeof(int), ctx->stream));
  HIPCHK(tp_set_radii(ctx->t, ctx->w.n, d_radii, ctx->w.flag_in, ctx->stream));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, ctx->w.flag_in, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (bad) {
    // leave no partial set behind: back to no collisions
    HIPCHK(hipMemsetAsync(ctx->t.rad, 0,
                          (kTpMaxPlanets + std::max<int64_t>(ctx->t.ntp, 1)) * sizeof(double),
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return GENGA_EINVAL;
  }
  return GENGA_OK;
}

int genga_collisions(genga_ctx* ctx, int64_t* h_tp, int32_t* h_planet, int64_t* h_step,
                     double* h_frac, double* h_xv, int64_t cap, int64_t* h_n) {
  if (!ctx || !h_n || cap < 0 || ctx->mode != GENGA_TEST) return GENGA_EINVAL;
  if (cap > 0 && (!h_tp || !h_planet || !h_step || !h_frac || !h_xv)) return GENGA_EINVAL;
  DevStat hs;
  int r = read_status(ctx, &hs);
  if (r != GENGA_OK) return r;
  // one slot per particle: more removals than particles (particles brought
  // back by genga_set_state and removed again) lose the later reports
  const int64_t total = (int64_t)hs.tp_removed;
  const int64_t n = std::min<int64_t>(total, ctx->t.ntp);
  std::vector<CollRec> recs((size_t)n);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(recs.data(), ctx->t.coll, (size_t)n * sizeof(CollRec),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  std::sort(recs.begin(), recs.end(), [](const CollRec& a, const CollRec& b) {
    return a.step != b.step ? a.step < b.step : a.tp < b.tp;
  });
  const int64_t wr = std::min(n, cap);
  for (int64_t k = 0; k < wr; ++k) {
    h_tp[k] = recs[k].tp;
    h_planet[k] = recs[k].planet;
    h_step[k] = recs[k].step;
    h_frac[k] = recs[k].frac;
    for (int q = 0; q < 6; ++q) h_xv[6 * k + q] = recs[k].xv[q];
  }
  *h_n = total;
  if (total > cap || total > n) return GENGA_EOVERFLOW;
  return status_from_flags(hs.flags);
}

int genga_events(genga_ctx* ctx, genga_event* h_ev, int64_t cap, int64_t* h_n) {
  if (!ctx || !h_n || cap < 0 || (cap > 0 && !h_ev) || ctx->mode == GENGA_TEST)
    return GENGA_EINVAL;
  DevStat hs;
  int r = read_status(ctx, &hs);
  if (r != GENGA_OK) return r;
  const bool bat = ctx->mode == GENGA_BATCH;
  unsigned long long cnt = 0;
  if (bat)
    HIPCHK(hipMemcpyAsync(&cnt, ctx->b.ev_cnt, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!bat) cnt = hs.ev_cnt;
  const int64_t have = std::min<int64_t>((int64_t)cnt, bat ? ctx->b.nb : (int64_t)ctx->w.ev_cap);
  std::vector<genga_event> ev((size_t)have);
  if (have > 0) {
    HIPCHK(hipMemcpyAsync(ev.data(), bat ? ctx->b.ev : ctx->w.ev, (size_t)have * sizeof(genga_event),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  std::sort(ev.begin(), ev.end(), [](const genga_event& a, const genga_event& b) {
    if (a.step != b.step) return a.step < b.step;
    if (a.sys != b.sys) return a.sys < b.sys;
    if (a.frac != b.frac) return a.frac < b.frac;
    return a.id_i < b.id_i;
  });
  for (int64_t k = 0; k < std::min(have, cap); ++k) h_ev[k] = ev[(size_t)k];
  *h_n = (int64_t)cnt;
  if ((int64_t)cnt > cap || (int64_t)cnt > have) return GENGA_EOVERFLOW;
  return status_from_flags(hs.flags);
}

int genga_bodies(genga_ctx* ctx, int32_t* h_id, int64_t cap, int32_t* h_nlive, double* h_U,
                 int sys_cap) {
  if (!ctx || ctx->mode == GENGA_TEST || cap < 0 || sys_cap < 0) return GENGA_EINVAL;
  if (ctx->mode == GENGA_MASSIVE) {
    if ((cap > 0 && !h_id) || (sys_cap > 0 && (!h_nlive || !h_U))) return GENGA_EINVAL;
    DevStat hs;
    int r = read_status(ctx, &hs);
    if (r != GENGA_OK) return r;
    const int n = ctx->w.n;
    std::vector<int32_t> ids((size_t)n);
    HIPCHK(hipMemcpyAsync(ids.data(), ctx->w.ids, ids.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < std::min<int64_t>(n, cap); ++q) h_id[q] = q < hs.nlive ? ids[q] : -1;
    if (sys_cap > 0) {
      h_nlive[0] = hs.nlive;
      h_U[0] = hs.U;
    }
    return cap < n || sys_cap < 1 ? GENGA_EOVERFLOW : GENGA_OK;
  }
  const BatchWs& b = ctx->b;
  if ((cap > 0 && !h_id) || (sys_cap > 0 && (!h_nlive || !h_U))) return GENGA_EINVAL;
  std::vector<BatchSysStat> ss((size_t)b.nsys);
  std::vector<int32_t> ids((size_t)b.nb), off((size_t)b.nsys + 1);
  HIPCHK(hipMemcpyAsync(ss.data(), b.ss, ss.size() * sizeof(BatchSysStat), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipMemcpyAsync(ids.data(), b.ids, ids.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipMemcpyAsync(off.data(), b.off, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int s = 0; s < b.nsys; ++s) {
    for (int r = off[s]; r < off[s + 1]; ++r)
      if (r < cap) h_id[r] = r - off[s] < ss[s].nlive ? ids[r] : -1;
    if (s < sys_cap) {
      h_nlive[s] = ss[s].nlive;
      h_U[s] = ss[s].U;
    }
  }
  return cap < b.nb || sys_cap < b.nsys ? GENGA_EOVERFLOW : GENGA_OK;
}

int genga_tune(genga_ctx* ctx, int nsteps, double* h_us, int cap, int* h_n, int* h_choice) {
  if (!ctx || ctx->mode != GENGA_BATCH || nsteps < 1 || cap < 0 || (cap > 0 && !h_us))
    return GENGA_EINVAL;
  const int r = batch_tune(ctx, nsteps);
  if (r != GENGA_OK) return r;
  for (int v = 0; v < std::min(cap, kBatchVariants); ++v) h_us[v] = ctx->tune_us[v];
  if (h_n) *h_n = kBatchVariants;
  if (h_choice) *h_choice = ctx->variant;
  return cap < kBatchVariants ? GENGA_EOVERFLOW : GENGA_OK;
}

const char* genga_tune_variant(int v) { return batch_variant_name(v); }

int genga_batch_set_variant(genga_ctx* ctx, int v) {
  if (!ctx || ctx->mode != GENGA_BATCH || !batch_variant_ok(ctx->b, v)) return GENGA_EINVAL;
  ctx->tuned = true;
  if (v != ctx->variant) {
    ctx->variant = v;
    if (ctx->g_batch) {
      (void)hipGraphExecDestroy(ctx->g_batch);
      ctx->g_batch = nullptr;
    }
  }
  return GENGA_OK;
}

int genga_batch_status(genga_ctx* ctx, int32_t* h_status, int64_t* h_steps, int cap) {
  if (!ctx || ctx->mode != GENGA_BATCH || cap < 0 || (cap > 0 && (!h_status || !h_steps)))
    return GENGA_EINVAL;
  std::vector<BatchSysStat> ss((size_t)ctx->b.nsys);
  HIPCHK(hipMemcpyAsync(ss.data(), ctx->b.ss, ss.size() * sizeof(BatchSysStat),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int s = 0; s < std::min(cap, ctx->b.nsys); ++s) {
    h_status[s] = status_from_flags(ss[s].flags & ~F_SYS_STOP);
    h_steps[s] = ss[s].steps;
  }
  return cap < ctx->b.nsys ? GENGA_EOVERFLOW : GENGA_OK;
}

// The encounter-free adjoint (K = 1), or the hybrid one: a batched context
// with encounters and no bodies leaving (no radii, rcut or rcut_sun).
static bool adj_hybrid(const genga_ctx* ctx) {
  return !ctx->p.encounter_free && !ctx->b.coll && ctx->b.rcut == 0.0 && ctx->b.rcut_sun == 0.0;
}
static bool adj_ok(const genga_ctx* ctx) {
  return ctx && ctx->mode == GENGA_BATCH && (ctx->p.encounter_free || adj_hybrid(ctx));
}

static size_t adj_ckpt_bytes(const genga_ctx* ctx, int64_t nsteps, int ckpt_every) {
  if (adj_hybrid(ctx)) return align256(hadj_ckpt_bytes(ctx->b.nb, (int)nsteps, ckpt_every));
  const int64_t C = (nsteps + ckpt_every - 1) / ckpt_every;
  return align256((size_t)C * 6 * (size_t)ctx->b.nb * sizeof(double));
}

size_t genga_adj_buffer_bytes(genga_ctx* ctx, int64_t nsteps, int ckpt_every) {
  if (!adj_ok(ctx) || nsteps < 1 || nsteps > INT_MAX || ckpt_every < 1) return 0;
  const int K = (int)std::min<int64_t>(ckpt_every, nsteps);
  if (adj_hybrid(ctx))
    return adj_ckpt_bytes(ctx, nsteps, ckpt_every) + hadj_work_bytes(ctx->b.nsys, K);
  return adj_ckpt_bytes(ctx, nsteps, ckpt_every) + adj_tape_bytes(ctx->b.nsys, ctx->sb, K);
}

int genga_adj_forward(genga_ctx* ctx, int64_t nsteps, int ckpt_every, void* d_buffer,
                      size_t buffer_bytes) {
  if (!adj_ok(ctx) || !d_buffer || ((uintptr_t)d_buffer & 255u) != 0) return GENGA_EINVAL;
  const size_t need = genga_adj_buffer_bytes(ctx, nsteps, ckpt_every);
  if (need == 0) return GENGA_EINVAL;
  if (buffer_bytes < need) return GENGA_ENOMEM;
  if (adj_hybrid(ctx))
    HIPCHK(hadj_forward(ctx->b, ctx->c, (int)nsteps, ckpt_every, (double*)d_buffer, ctx->stream));
  else
    HIPCHK(adj_forward(ctx->b, ctx->c, ctx->sb, (int)nsteps, ckpt_every, (double*)d_buffer,
                       ctx->stream));
  ctx->adj_ckpt = (double*)d_buffer;
  ctx->adj_bytes = buffer_bytes;
  ctx->adj_T = (int)nsteps;
  ctx->adj_K = ckpt_every;
  ctx->steps += nsteps;
  return GENGA_OK;
}

int genga_adj_backward(genga_ctx* ctx, const double* d_gxT, const double* d_gvT, double* d_gx0,
                       double* d_gv0, double* d_gm) {
  if (!adj_ok(ctx) || !ctx->adj_ckpt || !d_gxT || !d_gvT || !d_gx0 || !d_gv0 || !d_gm)
    return GENGA_EINVAL;
  const int T = ctx->adj_T, K = ctx->adj_K;
  double* tape = (double*)((char*)ctx->adj_ckpt + adj_ckpt_bytes(ctx, T, K));
  if (adj_hybrid(ctx))
    HIPCHK(hadj_backward(ctx->b, ctx->c, T, std::min(K, T), ctx->adj_ckpt, tape, d_gxT, d_gvT,
                         d_gx0, d_gv0, d_gm, ctx->stream));
  else
    HIPCHK(adj_backward(ctx->b, ctx->c, ctx->sb, T, std::min(K, T), ctx->adj_ckpt, tape, d_gxT,
                        d_gvT, d_gx0, d_gv0, d_gm, ctx->stream));
  return GENGA_OK;
}

const char* genga_strerror(int code) {
  switch (code) {
    case GENGA_OK: return "ok";
    case GENGA_EINVAL: return "invalid argument";
    case GENGA_EHIP: return "HIP runtime error";
    case GENGA_EOVERFLOW: return "list capacity exceeded";
    case GENGA_EKEPLER: return "Kepler iteration did not converge";
    case GENGA_EBS: return "Bulirsch-Stoer depth exhausted";
    case GENGA_EADJ_ENCOUNTER: return "pair inside the critical radius in the encounter-free adjoint";
    case GENGA_ENOMEM: return "workspace too small";
    case GENGA_EGROUP: return "encounter group too large";
    case GENGA_WSTOPPED: return "some systems stopped after a failed step (see genga_batch_status)";
    default: return "unknown error";
  }
}

int genga_destroy(genga_ctx* ctx) {
  if (!ctx) return GENGA_EINVAL;
  if (ctx->stream || ctx->cap) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->g_many) (void)hipGraphExecDestroy(ctx->g_many);
  if (ctx->g_batch) (void)hipGraphExecDestroy(ctx->g_batch);
  for (hipGraphExec_t g : ctx->g_rem)
    if (g) (void)hipGraphExecDestroy(g);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  delete ctx;
  return GENGA_OK;
}

size_t genga_accel_workspace_bytes(int n) {
  if (n < 1 || n > 65536) return 0;
  genga_params p;
  genga_params_default(&p);
  return massive_ws_bytes(n, accel_params(p));
}

int genga_accel(const genga_params* p, int n, const double* d_m, const double* d_x,
                const double* d_rc, double* d_acc, void* d_workspace, size_t ws_bytes,
                void* stream) {
  if (!params_ok(p) || n < 1 || n > 65536 || !d_m || !d_x || !d_acc || !d_workspace)
    return GENGA_EINVAL;
  if (!p->encounter_free && !d_rc) return GENGA_EINVAL;
  if (((uintptr_t)d_workspace & 255u) != 0) return GENGA_EINVAL;
  const genga_params q = accel_params(*p);
  if (ws_bytes < massive_ws_bytes(n, q)) return GENGA_ENOMEM;
  MassiveWs w;
  massive_carve(w, n, q, d_workspace);
  HIPCHK(accel_run(w, make_consts(q), d_m, d_x, d_rc, d_acc, (hipStream_t)stream));
  return GENGA_OK;
}

int genga_accel_noalloc(const genga_params* p, int n, const double* d_m, const double* d_x,
                        const double* d_rc, double* d_acc, void* stream) {
  if (!params_ok(p) || n < 1 || n > GENGA_ACCEL_NOALLOC_MAX || !d_m || !d_x || !d_acc)
    return GENGA_EINVAL;
  if (!p->encounter_free && !d_rc) return GENGA_EINVAL;
  HIPCHK(accel_noalloc_run(make_consts(accel_params(*p)), n, d_m, d_x, d_rc, d_acc,
                           (hipStream_t)stream));
  return GENGA_OK;
}

int genga_kepler(double mu, int64_t n, const double* d_x0, const double* d_v0, double dt,
                 double* d_x, double* d_v, int max_iter, int32_t* d_iters, void* stream) {
  if (n < 0 || !(mu > 0.0) || !std::isfinite(dt) || max_iter < 1) return GENGA_EINVAL;
  if (n > 0 && (!d_x0 || !d_v0 || !d_x || !d_v)) return GENGA_EINVAL;
  HIPCHK(op_kepler(mu, n, d_x0, d_v0, dt, d_x, d_v, max_iter, d_iters, (hipStream_t)stream));
  return GENGA_OK;
}

int genga_hermite(int64_t n, double dt, const double* d_q, double* d_out, void* stream) {
  if (n < 0 || !std::isfinite(dt)) return GENGA_EINVAL;
  if (n > 0 && (!d_q || !d_out)) return GENGA_EINVAL;
  HIPCHK(op_hermite(n, dt, d_q, d_out, (hipStream_t)stream));
  return GENGA_OK;
}

}  // extern "C"
