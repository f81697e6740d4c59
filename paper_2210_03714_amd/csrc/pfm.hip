// libpfm host runtime: the C ABI of include/pfm.h on top of the gfx950 kernels.
//
// A call of pfm_eval_batched validates on the host, lays out the workspace
// from the sizes alone, and enqueues the whole path: the per-instance plan
// (s or N) and route are decided on the device from ||A||_1, the kernels of
// every route are launched over all instances that may take it (the others
// return at once), and the squarings run as a fixed number of per-level
// launches followed by a persistent queue for any further levels
// (kern_sched.h).  Nothing is read back, so the call does not wait for the
// GPU (except to grow the workspace, or for the step count of an action on
// an instance above 512).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <string>
#include <vector>

#include "pfm.h"
#include "pfm_internal.h"
#include "pfm_tables.inc"
#include "kern_common.h"
#include "kern_lu.h"
#include "kern_misc.h"
#include "kern_solve.h"
#include "kern_square.h"
#include "kern_action.h"
#include "kern_mixed.h"
#include "kern_gj.h"
#include "kern_gj2.h"
#include "kern_large.h"
#include "kern_tri.h"
#include "kern_band.h"
#include "kern_sched.h"

using namespace pfm;
static_assert(kNCap == PFM_MAX_STEPS, "the device-side step cap is the documented one");
static_assert(kSCap == PFM_MAX_SQUARINGS, "the device-side squaring cap is the documented one");

// phases timed by pfm_profile: LU, solve+combine, squaring, store
constexpr int kNumPhases = 4;

struct pfm_ctx {
  int device = 0;
  size_t budget = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  int *d_err = nullptr;  // device-side error flags
  int num_cu = 0;
  // pinned host staging for descriptors, plans and task lists; the event
  // marks the last upload that reads it
  char *pin = nullptr;
  size_t pin_bytes = 0;
  hipEvent_t pin_ev = nullptr;
  bool pin_pending = false;
  // device buffer for per-level squaring task lists
  void *tasks = nullptr;
  size_t tasks_bytes = 0;
  // Gauss-Jordan route for diagonally dominant shifted matrices
  // (pfm_set_route(PFM_ROUTE_LU) disables it), and the size above which
  // action / complex instances may take the multi-workgroup route
  int gj = 1;
  int ln_min = kLnMin;
  // squaring levels launched one by one; the rest run from the persistent
  // queue (kern_sched.h)
  int sq_direct = 8;
  bool sched_explicit = false;  // set by pfm_set_schedule: a tuned schedule does not override it
  // the bytes (pointers, descriptors, lists, task lists) of the last upload
  // of pfm_eval_batched, valid while nothing else has written the workspace
  std::vector<char> up_key;
  bool up_valid = false;
  // autotuned policies per batch key (pfm_tune); force_policy >= 0 while
  // tuning
  std::map<uint64_t, int> tuned;
  int force_policy = -1;
  // hipGraph reuse of repeated launch sequences (pfm_set_graphs)
  bool graphs = true;
  uint64_t gsig = 0, gseen = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_captures = 0, graph_replays = 0;
  // optional phase timing (hipEvents on the caller's stream)
  bool prof = false;
  bool prof_pending = false;
  hipEvent_t pev[kNumPhases + 1] = {};
  double prof_ms[kNumPhases] = {};
  int prof_launches[kNumPhases] = {};
  int prof_calls = 0;
  int cur_launches[kNumPhases] = {};
  // where the last pfm_eval_batched call left its factorisations
  // (pfm_lu_factors); cleared whenever another call reuses the workspace
  std::vector<InstDesc> fac_desc;
  int fac_nterms = 0;
  bool fac_mixed = false;
  const double *fac_wsd = nullptr;
  const int *fac_wsi = nullptr;
  const PlanRec *fac_plan = nullptr;
  std::string err;
};

// ---------------------------------------------------------------------------
// Allocation-free scratch.  pfm_tri_action_noalloc keeps its descriptors,
// plans, factors, vectors and checkpoints in this fixed array instead of the
// context's workspace.  The name is a host-side stand-in, never a device
// address: host code uses only the address hipGetSymbolAddress returned for
// the device (g_scratch_dev), looked up once per device by pfm_create with
// that device current.  Every call on a device shares that device's copy.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)PFM_NOALLOC_MAX_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

int set_err(pfm_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int set_err(pfm_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

#define HIP_TRY(ctx, call)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_err(ctx, PFM_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

inline bool T_want_phi(int f) { return f != PFM_LOG1M && (f & (PFM_PHI1 | PFM_PHI2)); }

// table index of a single function bit (PFM_EXP 0, PFM_PHI1 1, PFM_LOG1M 2,
// PFM_PHI2 3)
inline int func_index(int f) { return f == PFM_EXP ? 0 : (f == PFM_PHI1 ? 1 : (f == PFM_LOG1M ? 2 : 3)); }

// a function mask pfm_eval_batched accepts: PFM_LOG1M alone, or a nonempty
// combination of PFM_EXP, PFM_PHI1 and PFM_PHI2
inline bool valid_mask(int f) { return f == PFM_LOG1M || (f > 0 && (f & ~(PFM_EXP | PFM_PHI1 | PFM_PHI2)) == 0); }

const PfmSetEntry *find_set(int m, int func) {
  for (int i = 0; i < kPfmNumSets; ++i)
    if (kPfmSets[i].m == m && kPfmSets[i].func == func) return &kPfmSets[i];
  return nullptr;
}

// eps(x) = sum_k d_k x^k (§3), Horner in extended precision; all d_k >= 0.
long double bound_eval(const PfmSetEntry *e, long double x) {
  long double s = 0.0L;
  for (int k = PFM_KBOUND - 1; k >= 0; --k) s = s * x + (long double)e->d[k];
  return s;
}

double theta_of(const PfmSetEntry *e, double tol) {
  double cmax = 0.0;
  for (int k = 0; k < e->nterms; ++k) cmax = std::max(cmax, std::hypot(e->c_re[k], e->c_im[k]));
  long double lo = 0.0L, hi = 0.9L / (long double)cmax;
  if (bound_eval(e, hi) <= tol) return (double)hi;
  for (int it = 0; it < 200; ++it) {
    const long double mid = 0.5L * (lo + hi);
    if (bound_eval(e, mid) <= (long double)tol) lo = mid; else hi = mid;
  }
  double v = (double)lo;
  if ((long double)v > lo) v = std::nextafter(v, 0.0);
  return v;
}

// The rounding floor of the round-off form (§4.3): a scaled step's result
// carries rounding of about (sum_k |w_k| + |d1| + |d2|) θ u (u = 2^-53), which
// the cancellation in the sum does not remove, so a tolerance below it cannot
// be met.  It is below 1e-14 for the partial-fraction sets, about 6e-13 for
// the hybrid set m = 10 at 1e-12, and about 2e-10 for R*10 (m = 110).
double rounding_floor(const PfmSetEntry *e, double theta) {
  if (!e) return 0.0;
  long double s = fabsl((long double)e->poly[0]) + fabsl((long double)e->poly[1]);
  for (int k = 0; k < e->nterms; ++k) s += (e->pair ? 2.0L : 1.0L) * (long double)std::hypot(e->w_re[k], e->w_im[k]);
  return (double)(s * (long double)theta * 0x1p-53L);
}

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
// user arrays are read and written one binary64 element (or half of a
// complex one) at a time: their addresses must be multiples of 8
inline bool misaligned(const void *p) { return ((uintptr_t)p & 7) != 0; }

// Pinned staging area of at least `bytes`; waits until the previous upload
// that read it has executed.
int staging(pfm_ctx *ctx, size_t bytes, char **out) {
  if (ctx->pin_pending) {
    HIP_TRY(ctx, hipEventSynchronize(ctx->pin_ev));
    ctx->pin_pending = false;
  }
  if (bytes > ctx->pin_bytes) {
    if (ctx->pin) HIP_TRY(ctx, hipHostFree(ctx->pin));
    ctx->pin = nullptr;
    ctx->pin_bytes = 0;
    const size_t nb = std::max<size_t>(bytes, 1 << 20);
    HIP_TRY(ctx, hipHostMalloc((void **)&ctx->pin, nb, hipHostMallocDefault));
    ctx->pin_bytes = nb;
  }
  *out = ctx->pin;
  return PFM_OK;
}

int prof_harvest(pfm_ctx *ctx) {
  if (!ctx->prof_pending) return PFM_OK;
  HIP_TRY(ctx, hipEventSynchronize(ctx->pev[kNumPhases]));
  for (int p = 0; p < kNumPhases; ++p) {
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->pev[p], ctx->pev[p + 1]));
    ctx->prof_ms[p] += ms;
    ctx->prof_launches[p] += ctx->cur_launches[p];
  }
  ctx->prof_calls++;
  ctx->prof_pending = false;
  return PFM_OK;
}

// Policies the autotuner chooses between: a route policy and a squaring
// schedule (policy index = route + kNumRoutePolicies * schedule).
struct Policy {
  int gj;      // single-workgroup Gauss-Jordan route for dominant real full matrices
  int ln_min;  // action / complex instances above this size may take the multi-workgroup route
};
constexpr Policy kPolicies[] = {{1, kLnMin}, {0, kLnMin}, {1, 512}, {0, 512}};
constexpr int kNumRoutePolicies = 4;
// squaring levels launched one by one before the persistent queue takes the
// rest: 8 (enough for ||A||_1 up to 2^8 θ), or 0 (the queue runs them all)
constexpr int kSqDirect[] = {8, 0};
constexpr int kNumSchedules = 2;
// smallest npad whose product tiles are 128 x 128 (else 64 x 64)
constexpr int kTile128Min[] = {256, 1 << 30};
constexpr int kNumTiles = 2;
// Gauss-Jordan pivot block of npad = 256 instances: 128 (gj2_inv_kernel,
// two passes over the matrix) or 64 (gj_inv_kernel, four passes)
constexpr int kGjBlock[] = {128, 64};
constexpr int kNumGjBlocks = 2;
constexpr int kNumPolicies = kNumRoutePolicies * kNumSchedules * kNumTiles * kNumGjBlocks;

// Tuning key of a batch: mode, complex, precision, size bucket of its
// largest real dimension (2n for complex), batch-size bucket.
uint64_t batch_key(bool action, bool emb, bool mixed, int batch, const pfm_problem *probs) {
  int nmax = 0;
  for (int i = 0; i < batch; ++i) nmax = std::max(nmax, emb ? 2 * probs[i].n : probs[i].n);
  const int sb = nmax <= 64 ? 0 : nmax <= 128 ? 1 : nmax <= 256 ? 2 : nmax <= 512 ? 3 : 4;
  const int bb = batch <= 1 ? 0 : batch <= 7 ? 1 : batch <= 63 ? 2 : 3;
  return (uint64_t)action | ((uint64_t)emb << 1) | ((uint64_t)mixed << 2) | ((uint64_t)sb << 4) |
         ((uint64_t)bb << 8);
}

inline void prof_mark(pfm_ctx *ctx, int idx, hipStream_t stream) {
  if (ctx->prof) (void)hipEventRecord(ctx->pev[idx], stream);
}

// The device addresses of `scratch`, one per device (see above).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;             // guards the table and the host descriptor staging below
char *g_scratch_dev[kMaxDevices] = {};
// host-side descriptors of the allocation-free call (static, so that no call
// allocates); hipMemcpyAsync from this pageable memory stages it before it
// returns, so the next call may overwrite it
TriDesc g_noalloc_desc[PFM_NOALLOC_MAX_BATCH];

// Resolve the device address of `scratch` for the current device.
int scratch_resolve(int device) {
  if (device < 0 || device >= kMaxDevices) return PFM_ERR_INVALID;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return PFM_OK;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PFM_ERR_HIP;
  g_scratch_dev[device] = (char *)ptr;
  return PFM_OK;
}

}  // namespace

extern "C" {

int pfm_set_route(pfm_ctx *ctx, int route) {
  if (!ctx) return PFM_ERR_INVALID;
  if (route != PFM_ROUTE_AUTO && route != PFM_ROUTE_LU)
    return set_err(ctx, PFM_ERR_INVALID, "pfm_set_route: unknown route %d", route);
  ctx->gj = route == PFM_ROUTE_AUTO;
  ctx->ln_min = route == PFM_ROUTE_AUTO ? kLnMin : 512;
  return PFM_OK;
}

int pfm_set_schedule(pfm_ctx *ctx, int direct_levels) {
  if (!ctx) return PFM_ERR_INVALID;
  if (direct_levels < 0 || direct_levels > PFM_MAX_SQUARINGS)
    return set_err(ctx, PFM_ERR_INVALID, "pfm_set_schedule: %d levels not in [0, %d]", direct_levels,
                   PFM_MAX_SQUARINGS);
  ctx->sq_direct = direct_levels;
  ctx->sched_explicit = true;
  return PFM_OK;
}

int pfm_profile(pfm_ctx *ctx, int enable) {
  if (!ctx) return PFM_ERR_INVALID;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (enable && !ctx->pev[0])
    for (int p = 0; p <= kNumPhases; ++p) HIP_TRY(ctx, hipEventCreate(&ctx->pev[p]));
  int rc = prof_harvest(ctx);
  if (rc) return rc;
  ctx->prof = enable != 0;
  for (int p = 0; p < kNumPhases; ++p) { ctx->prof_ms[p] = 0.0; ctx->prof_launches[p] = 0; }
  ctx->prof_calls = 0;
  return PFM_OK;
}

int pfm_profile_read(pfm_ctx *ctx, double *ms, int *launches, int *calls) {
  if (!ctx || !ms) return PFM_ERR_INVALID;
  int rc = prof_harvest(ctx);
  if (rc) return rc;
  for (int p = 0; p < kNumPhases; ++p) {
    ms[p] = ctx->prof_ms[p];
    if (launches) launches[p] = ctx->prof_launches[p];
  }
  if (calls) *calls = ctx->prof_calls;
  return PFM_OK;
}

size_t pfm_workspace_bytes(int f, int m, int prec, int dtype, int batch, const pfm_problem *probs) {
  if (!valid_mask(f) || f == PFM_LOG1M || batch < 1 || !probs) return 0;
  const PfmSetEntry *ee = find_set(m, 0), *ep = find_set(m, 1);
  if (!ee || (!ep && (f & (PFM_PHI1 | PFM_PHI2))) || ((f & PFM_PHI2) && !find_set(m, 3))) return 0;
  const int64_t rbufs = (f & PFM_PHI2) ? 6 : 4;
  const bool cplx = dtype == PFM_C128, pairs = ee->pair != 0, mixed = prec == PFM_MIXED;
  const bool emb = cplx || pairs;
  const bool phi = (f & PFM_PHI1) != 0;
  if (prec != PFM_FP64 && prec != PFM_MIXED) return 0;
  if (dtype != PFM_R64 && dtype != PFM_C128) return 0;
  const bool act = probs[0].p > 0;
  if (mixed && (cplx || pairs || act)) return 0;
  const int64_t nterms = pairs ? (int64_t)(cplx ? 2 : 1) * (1 + (phi ? 1 : 0)) : ee->nterms;
  int64_t d = 4096 / 8, ints = 0;
  for (int i = 0; i < batch; ++i) {
    const pfm_problem &P = probs[i];
    if (P.n < 1 || P.p < 0 || (P.p > 0) != act) return 0;
    const int64_t nk = emb ? 2 * (int64_t)P.n : P.n;
    if (nk > 512 && (mixed || pairs || nk > kLargeMax || P.p > 64)) return 0;
    const int64_t np = (nk + 63) / 64 * 64, nn = np * np;
    const bool large = nk > 512;
    const bool may_ln = large || (!mixed && !pairs && nk > kLnMin && (act || emb));
    d += nterms * nn + rbufs * nn + 6 * 64;
    if (may_ln) {
      d += nterms * ln_stride((int)np);
      if (P.p > 0) d += 2 * ln_vchain((int)np, P.p) + (int64_t)ln_ks((int)nk) * np * ln_pp(P.p);
    }
    if (!large) d += nterms * 2 * (np / 16) * 256;
    if (emb || mixed) d += std::max(nk, np) * np;
    ints += large ? 0 : 2 * nterms * np + 128;
    // plan, descriptor, list entries and squaring-queue entries
    d += (sizeof(PlanRec) + sizeof(InstDesc) + 4 * sizeof(int) + 16 + 7) / 8;
  }
  return (size_t)(d * 8 + ints * 4 + 2 * (kSCap + 2) * 8 + 16 * 256 + 4096);
}

const char *pfm_version(void) { return "pfm 0.2 (gfx950)"; }

int pfm_create(pfm_ctx **out, int device, size_t budget) {
  if (!out) return PFM_ERR_INVALID;
  *out = nullptr;
  pfm_ctx *ctx = new pfm_ctx();
  ctx->device = device;
  ctx->budget = budget;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) { delete ctx; return PFM_ERR_HIP; }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) { delete ctx; return PFM_ERR_HIP; }
  ctx->num_cu = prop.multiProcessorCount;
  // library set-up for this device: the address of its allocation-free
  // scratch array (pfm_tri_action_noalloc), with the device current
  if (scratch_resolve(device) != PFM_OK) { delete ctx; return PFM_ERR_HIP; }
  e = hipMalloc(&ctx->d_err, 64);
  if (e != hipSuccess) { delete ctx; return PFM_ERR_HIP; }
  e = hipMemset(ctx->d_err, 0, 64);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->pin_ev, hipEventDisableTiming);
  if (e != hipSuccess) { (void)hipFree(ctx->d_err); delete ctx; return PFM_ERR_HIP; }
  *out = ctx;
  return PFM_OK;
}

int pfm_destroy(pfm_ctx *ctx) {
  if (!ctx) return PFM_ERR_INVALID;
  (void)hipSetDevice(ctx->device);
  for (int p = 0; p <= kNumPhases; ++p)
    if (ctx->pev[p]) (void)hipEventDestroy(ctx->pev[p]);
  if (ctx->pin_ev) {
    (void)hipEventSynchronize(ctx->pin_ev);
    (void)hipEventDestroy(ctx->pin_ev);
  }
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->tasks) (void)hipFree(ctx->tasks);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  if (ctx->d_err) (void)hipFree(ctx->d_err);
  delete ctx;
  return PFM_OK;
}

const char *pfm_last_error(const pfm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int pfm_coeffs(int f, int m, int *n_terms, double *c_re, double *c_im, double *w_re, double *w_im,
               double *a0, int *order, int *is_pair) {
  if (f != PFM_EXP && f != PFM_PHI1 && f != PFM_LOG1M && f != PFM_PHI2) return PFM_ERR_INVALID;
  const PfmSetEntry *e = find_set(m, func_index(f));
  if (!e) return PFM_ERR_UNSUPPORTED;
  if (n_terms) *n_terms = e->nterms;
  for (int k = 0; k < e->nterms; ++k) {
    if (c_re) c_re[k] = e->c_re[k];
    if (c_im) c_im[k] = e->c_im[k];
    if (w_re) w_re[k] = e->w_re[k];
    if (w_im) w_im[k] = e->w_im[k];
  }
  if (a0) *a0 = e->a0;
  if (order) *order = e->order;
  if (is_pair) *is_pair = e->pair;
  return PFM_OK;
}

int pfm_poly(int f, int m, double *d1, double *d2) {
  if (f != PFM_EXP && f != PFM_PHI1 && f != PFM_LOG1M && f != PFM_PHI2) return PFM_ERR_INVALID;
  const PfmSetEntry *e = find_set(m, func_index(f));
  if (!e) return PFM_ERR_UNSUPPORTED;
  if (d1) *d1 = e->poly[0];
  if (d2) *d2 = e->poly[1];
  return PFM_OK;
}

int pfm_theta(int f, int m, double tol, double *theta) {
  if (!theta || !(tol > 0.0 && tol < 1.0)) return PFM_ERR_INVALID;
  if (f == PFM_LOG1M) {  // on its own set, without the exponential
    const PfmSetEntry *el = find_set(m, 2);
    if (!el) return PFM_ERR_UNSUPPORTED;
    *theta = theta_of(el, tol);
    return PFM_OK;
  }
  if (!valid_mask(f)) return PFM_ERR_INVALID;
  // phi1 always carries the exponential approximant too (its doubling and its
  // recurrence apply e^B), and phi2 carries both (its doubling squares phi1),
  // so θ is the smallest of those involved.
  const PfmSetEntry *ee = find_set(m, 0);
  const PfmSetEntry *ep = find_set(m, 1);
  const PfmSetEntry *eq = find_set(m, 3);
  if (!ee || (!ep && (f & (PFM_PHI1 | PFM_PHI2))) || (!eq && (f & PFM_PHI2))) return PFM_ERR_UNSUPPORTED;
  double th = theta_of(ee, tol);
  if (f & (PFM_PHI1 | PFM_PHI2)) th = std::min(th, theta_of(ep, tol));
  if (f & PFM_PHI2) th = std::min(th, theta_of(eq, tol));
  *theta = th;
  return PFM_OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Tridiagonal and banded actions: host set-up shared by pfm_tri_action,
// pfm_band_action and the allocation-free pfm_tri_action_noalloc.  Neither
// reads anything back from the device: the plan kernels cap N themselves
// (PFM_NOT_COMPUTED above kNCap), so a call only enqueues work.
// ---------------------------------------------------------------------------

// Coefficients of a tridiagonal / banded call: a real shift set (m = 4, 5,
// 8, or 10, the hybrid set of §4.3 for the exponential only), θ(f, m, tol)
// and the order of the approximation.
int sparse_terms(pfm_ctx *ctx, const char *what, int f, int m, double tol, TriTerms *T, double *theta,
                 int *order) {
  const PfmSetEntry *ee = find_set(m, 0), *ep = find_set(m, 1);
  if (!ee || (!ep && (f & PFM_PHI1))) return set_err(ctx, PFM_ERR_UNSUPPORTED, "no coefficient set for m = %d", m);
  const bool hybrid = ee->poly[0] != 0.0 || ee->poly[1] != 0.0;
  if (ee->pair || !(ee->nterms == 4 || ee->nterms == 5 || ee->nterms == 8 || (hybrid && ee->nterms == 10)))
    return set_err(ctx, PFM_ERR_UNSUPPORTED, "the %s path takes the real shift sets (m = 4, 5, 8, 10)", what);
  if (hybrid && f != PFM_EXP)
    return set_err(ctx, PFM_ERR_UNSUPPORTED, "the hybrid set is provided for the exponential only");
  const int rc = pfm_theta(f, m, tol, theta);
  if (rc) return set_err(ctx, rc, "theta failed");
  {
    const double fl = std::max(rounding_floor(ee, *theta), (f & PFM_PHI1) ? rounding_floor(ep, *theta) : 0.0);
    if (tol < fl)
      return set_err(ctx, PFM_ERR_UNSUPPORTED, "tol %g is below the rounding floor %.2g of the m = %d set", tol, fl, m);
  }
  memset(T, 0, sizeof *T);
  T->nterms = ee->nterms;
  T->nf = 0;
  if (f & PFM_EXP) T->fn[T->nf++] = 0;
  if (f & PFM_PHI1) T->fn[T->nf++] = 1;
  T->a0e = ee->a0;
  T->a0p = ep ? ep->a0 : 0.0;
  for (int k = 0; k < T->nterms; ++k) {
    T->c[k] = ee->c_re[k];
    T->we[k] = ee->w_re[k];
    T->wp[k] = ep ? ep->w_re[k] : 0.0;
  }
  T->d1 = ee->poly[0];
  T->d2 = ee->poly[1];
  *order = ee->order;
  return PFM_OK;
}

int tri_validate(pfm_ctx *ctx, int f, double tol, int batch, const pfm_tri_problem *probs) {
  if (f & PFM_PHI2) return set_err(ctx, PFM_ERR_UNSUPPORTED, "phi2 is provided for dense full matrices");
  if (f < 1 || f > 3) return set_err(ctx, PFM_ERR_INVALID, "bad function mask %d", f);
  if (!(tol > 0.0 && tol < 1.0)) return set_err(ctx, PFM_ERR_INVALID, "tol must lie in (0,1)");
  if (batch < 1 || !probs) return set_err(ctx, PFM_ERR_INVALID, "empty batch");
  for (int i = 0; i < batch; ++i) {
    const pfm_tri_problem &P = probs[i];
    if (P.d < 1 || P.d > PFM_TRI_MAX_D || P.p < 1 || P.p > PFM_TRI_MAX_P)
      return set_err(ctx, PFM_ERR_INVALID, "problem %d: bad d or p", i);
    if (!P.dd || !P.V || (P.d > 1 && (!P.dl || !P.du)))
      return set_err(ctx, PFM_ERR_INVALID, "problem %d: null diagonal or V", i);
    if (P.ldv < P.p || P.ldf < P.p) return set_err(ctx, PFM_ERR_INVALID, "problem %d: ldv or ldf < p", i);
    if ((f & PFM_EXP) && !P.F_exp) return set_err(ctx, PFM_ERR_INVALID, "problem %d: F_exp null", i);
    if ((f & PFM_PHI1) && !P.F_phi1) return set_err(ctx, PFM_ERR_INVALID, "problem %d: F_phi1 null", i);
    if (misaligned(P.dl) || misaligned(P.dd) || misaligned(P.du) || misaligned(P.V) || misaligned(P.F_exp) ||
        misaligned(P.F_phi1))
      return set_err(ctx, PFM_ERR_INVALID, "problem %d: an array is not 8-byte aligned", i);
  }
  return PFM_OK;
}

// Descriptor of one tridiagonal instance; its B and factors take the next
// doubles of the workspace from *dofs.  d <= kTsMaxD: its steps run in
// tri_scan_kernel, whose next workgroups (*sgs) it takes; else in
// tri_steps_kernel, whose next waves (*waves) it takes, with its vectors and
// checkpoints in the workspace as well.
void tri_desc(const pfm_tri_problem &P, const TriTerms &T, double theta, int64_t *dofs, int64_t *waves,
              int64_t *sgs, TriDesc *D) {
  memset(D, 0, sizeof *D);
  D->dl = P.dl;
  D->dd = P.dd;
  D->du = P.du;
  D->V = P.V;
  D->Fe = P.F_exp;
  D->Fp = P.F_phi1;
  D->ldv = P.ldv;
  D->ldf = P.ldf;
  D->d = P.d;
  D->p = P.p;
  D->theta = theta;
  const int64_t d = P.d, p = P.p, nch = (d + kTriL - 1) / kTriL;
  D->b_off = *dofs; *dofs += align_up(3 * d, 64);
  D->f_off = *dofs; *dofs += align_up(3 * d * T.nterms, 64);
  D->wave0 = (int32_t)*waves;
  D->sg0 = (int32_t)*sgs;
  if (d <= kTsMaxD) {
    D->nsg = T.nf * (int32_t)((p + kTsW - 1) / kTsW);
    *sgs += D->nsg;
    return;
  }
  D->v_off = *dofs; *dofs += align_up((int64_t)T.nf * 3 * d * p, 64);
  D->c_off = *dofs; *dofs += align_up((int64_t)T.nf * nch * T.nterms * p, 64);
  D->nwaves = T.nf * (int32_t)((p + 63) / 64);
  *waves += D->nwaves;
}

// Enqueue a tridiagonal call whose descriptors are (or will be, earlier on
// the stream) at d_desc: plan, factorisations, the N steps, the info records.
int tri_launch(pfm_ctx *ctx, const TriTerms &T, int order, int batch, const TriDesc *d_desc, PlanRec *d_plan,
               double *wsd, int64_t waves, int64_t sgs, pfm_info *info, int force_plan, hipStream_t stream) {
  hipLaunchKernelGGL(tri_plan_kernel, dim3(batch), dim3(256), 0, stream, d_desc, d_plan, force_plan);
  HIP_TRY(ctx, hipGetLastError());
  {
    int rcp = prof_harvest(ctx);
    if (rcp) return rcp;
  }
  // phase timing (pfm_profile): 0 the factorisations, 1 the N steps
  for (int ph = 0; ph < kNumPhases; ++ph) ctx->cur_launches[ph] = 0;
  prof_mark(ctx, 0, stream);
  const int nfac = batch * T.nterms;
  hipLaunchKernelGGL(tri_factor_kernel, dim3((nfac + 63) / 64), dim3(64), 0, stream, d_desc, d_plan, batch, T,
                     wsd);
  ctx->cur_launches[0]++;
  prof_mark(ctx, 1, stream);
#define PFM_TRI_STEPS(NT, PHI, HYB)                                                                            \
  do {                                                                                                         \
    if (sgs)                                                                                                   \
      hipLaunchKernelGGL((tri_scan_kernel<NT, PHI, HYB>), dim3((unsigned)align_up(sgs, 8)), dim3(64 * kTsW), 0, \
                         stream, d_desc, batch, d_plan, T, (const double *)wsd, (int)sgs);                      \
    if (waves)                                                                                                 \
      hipLaunchKernelGGL((tri_steps_kernel<NT, PHI, HYB>), dim3((unsigned)waves), dim3(64), 0, stream, d_desc, \
                         batch, d_plan, T, (const double *)wsd, wsd);                                          \
  } while (0)
  const bool hybrid = T.d1 != 0.0 || T.d2 != 0.0;
  const bool tri_phi = T.fn[0] == 1 || (T.nf > 1 && T.fn[1] == 1);
  if (hybrid) {
    PFM_TRI_STEPS(10, false, true);
  } else if (T.nterms == 4) {
    if (tri_phi) PFM_TRI_STEPS(4, true, false);
    else PFM_TRI_STEPS(4, false, false);
  } else if (T.nterms == 5) {
    if (tri_phi) PFM_TRI_STEPS(5, true, false);
    else PFM_TRI_STEPS(5, false, false);
  } else {
    if (tri_phi) PFM_TRI_STEPS(8, true, false);
    else PFM_TRI_STEPS(8, false, false);
  }
#undef PFM_TRI_STEPS
  ctx->cur_launches[1]++;
  prof_mark(ctx, 2, stream);
  prof_mark(ctx, 3, stream);
  if (info)
    hipLaunchKernelGGL(tri_info_kernel, dim3((batch + 255) / 256), dim3(256), 0, stream, d_desc, d_plan,
                       (InfoRec *)info, batch, order);
  prof_mark(ctx, 4, stream);
  if (ctx->prof) ctx->prof_pending = true;
  HIP_TRY(ctx, hipGetLastError());
  return PFM_OK;
}

// Grow the context's workspace to at least `need` bytes.
int ws_reserve(pfm_ctx *ctx, int64_t need, hipStream_t stream) {
  ctx->up_valid = false;  // this call writes its descriptors at the workspace's start
  ctx->fac_desc.clear();
  if (ctx->budget && (size_t)need > ctx->budget)
    return set_err(ctx, PFM_ERR_BUDGET, "workspace %lld bytes exceeds budget %zu", (long long)need, ctx->budget);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if ((size_t)need > ctx->ws_bytes) {
    if (ctx->ws) {
      HIP_TRY(ctx, hipStreamSynchronize(stream));
      HIP_TRY(ctx, hipFree(ctx->ws));
      ctx->ws = nullptr;
      ctx->ws_bytes = 0;
    }
    HIP_TRY(ctx, hipMalloc(&ctx->ws, (size_t)need));
    ctx->ws_bytes = (size_t)need;
  }
  return PFM_OK;
}

// Copy `bytes` of descriptors to d_dst through the pinned staging area; the
// staging is reused only after this upload has executed.
int upload_desc(pfm_ctx *ctx, void *d_dst, const void *src, size_t bytes, hipStream_t stream) {
  char *pin = nullptr;
  int rcs = staging(ctx, bytes, &pin);
  if (rcs) return rcs;
  memcpy(pin, src, bytes);
  HIP_TRY(ctx, hipMemcpyAsync(d_dst, pin, bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(ctx, hipEventRecord(ctx->pin_ev, stream));
  ctx->pin_pending = true;
  return PFM_OK;
}

}  // namespace

extern "C" {

int pfm_tri_action(pfm_ctx *ctx, int f, int m, double tol, int batch, const pfm_tri_problem *probs,
                   pfm_info *info, int force_plan, pfm_stream_t stream_) {
  if (!ctx) return PFM_ERR_INVALID;
  int rc = tri_validate(ctx, f, tol, batch, probs);
  if (rc) return rc;
  TriTerms T;
  double theta;
  int order;
  rc = sparse_terms(ctx, "tridiagonal", f, m, tol, &T, &theta, &order);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  std::vector<TriDesc> desc(batch);
  int64_t dofs = 0, waves = 0, sgs = 0;
  for (int i = 0; i < batch; ++i) {
    tri_desc(probs[i], T, theta, &dofs, &waves, &sgs, &desc[i]);
    if (waves > (int64_t)1 << 30 || sgs > (int64_t)1 << 30)
      return set_err(ctx, PFM_ERR_INVALID, "too many columns in one call");
  }
  const int64_t desc_bytes = align_up((int64_t)batch * sizeof(TriDesc), 256);
  const int64_t plan_bytes = align_up((int64_t)batch * sizeof(PlanRec), 256);
  rc = ws_reserve(ctx, desc_bytes + plan_bytes + dofs * 8, stream);
  if (rc) return rc;
  char *base = (char *)ctx->ws;
  TriDesc *d_desc = (TriDesc *)base;
  PlanRec *d_plan = (PlanRec *)(base + desc_bytes);
  double *wsd = (double *)(base + desc_bytes + plan_bytes);
  rc = upload_desc(ctx, d_desc, desc.data(), batch * sizeof(TriDesc), stream);
  if (rc) return rc;
  return tri_launch(ctx, T, order, batch, d_desc, d_plan, wsd, waves, sgs, info, force_plan, stream);
}

int pfm_tri_action_noalloc(pfm_ctx *ctx, int f, int m, double tol, int batch, const pfm_tri_problem *probs,
                           pfm_info *info, int force_plan, pfm_stream_t stream_) {
  if (!ctx) return PFM_ERR_INVALID;
  int rc = tri_validate(ctx, f, tol, batch, probs);
  if (rc) return rc;
  if (batch > PFM_NOALLOC_MAX_BATCH)
    return set_err(ctx, PFM_ERR_BUDGET, "batch %d exceeds the allocation-free limit of %d instances", batch,
                   PFM_NOALLOC_MAX_BATCH);
  TriTerms T;
  double theta;
  int order;
  rc = sparse_terms(ctx, "tridiagonal", f, m, tol, &T, &theta, &order);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  char *base = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch_dev[ctx->device] : nullptr;
  if (!base) return set_err(ctx, PFM_ERR_HIP, "the scratch array of device %d was not resolved", ctx->device);
  const int64_t desc_bytes = align_up((int64_t)batch * sizeof(TriDesc), 256);
  const int64_t plan_bytes = align_up((int64_t)batch * sizeof(PlanRec), 256);
  int64_t dofs = 0, waves = 0, sgs = 0;
  for (int i = 0; i < batch; ++i) {
    tri_desc(probs[i], T, theta, &dofs, &waves, &sgs, &g_noalloc_desc[i]);
    if (waves > (int64_t)1 << 30 || sgs > (int64_t)1 << 30)
      return set_err(ctx, PFM_ERR_INVALID, "too many columns in one call");
  }
  const int64_t need = desc_bytes + plan_bytes + dofs * 8;
  if ((size_t)need > kScratchBytes)
    return set_err(ctx, PFM_ERR_BUDGET,
                   "the call needs %lld bytes of scratch, more than the allocation-free limit of %zu",
                   (long long)need, kScratchBytes);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  TriDesc *d_desc = (TriDesc *)base;
  PlanRec *d_plan = (PlanRec *)(base + desc_bytes);
  double *wsd = (double *)(base + desc_bytes + plan_bytes);
  HIP_TRY(ctx, hipMemcpyAsync(d_desc, g_noalloc_desc, batch * sizeof(TriDesc), hipMemcpyHostToDevice, stream));
  return tri_launch(ctx, T, order, batch, d_desc, d_plan, wsd, waves, sgs, info, force_plan, stream);
}

int pfm_band_action(pfm_ctx *ctx, int f, int m, double tol, int b, int batch, const pfm_band_problem *probs,
                    pfm_info *info, int force_plan, pfm_stream_t stream_) {
  if (!ctx) return PFM_ERR_INVALID;
  if (f & PFM_PHI2) return set_err(ctx, PFM_ERR_UNSUPPORTED, "phi2 is provided for dense full matrices");
  if (f < 1 || f > 3) return set_err(ctx, PFM_ERR_INVALID, "bad function mask %d", f);
  if (!(tol > 0.0 && tol < 1.0)) return set_err(ctx, PFM_ERR_INVALID, "tol must lie in (0,1)");
  if (b < 1 || b > PFM_BAND_MAX_B) return set_err(ctx, PFM_ERR_INVALID, "half-bandwidth b = %d not in [1, %d]", b,
                                                  PFM_BAND_MAX_B);
  if (batch < 1 || !probs) return set_err(ctx, PFM_ERR_INVALID, "empty batch");
  for (int i = 0; i < batch; ++i) {
    const pfm_band_problem &P = probs[i];
    if (P.d < 1 || P.d > PFM_TRI_MAX_D || P.p < 1 || P.p > PFM_TRI_MAX_P)
      return set_err(ctx, PFM_ERR_INVALID, "problem %d: bad d or p", i);
    if (!P.bands || !P.V) return set_err(ctx, PFM_ERR_INVALID, "problem %d: null bands or V", i);
    if (P.ldv < P.p || P.ldf < P.p) return set_err(ctx, PFM_ERR_INVALID, "problem %d: ldv or ldf < p", i);
    if ((f & PFM_EXP) && !P.F_exp) return set_err(ctx, PFM_ERR_INVALID, "problem %d: F_exp null", i);
    if ((f & PFM_PHI1) && !P.F_phi1) return set_err(ctx, PFM_ERR_INVALID, "problem %d: F_phi1 null", i);
    if (misaligned(P.bands) || misaligned(P.V) || misaligned(P.F_exp) || misaligned(P.F_phi1))
      return set_err(ctx, PFM_ERR_INVALID, "problem %d: an array is not 8-byte aligned", i);
  }
  TriTerms T;
  double theta;
  int order;
  int rc = sparse_terms(ctx, "banded", f, m, tol, &T, &theta, &order);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  std::vector<BandDesc> desc(batch);
  int64_t dofs = 0;
  int64_t waves = 0, sgs = 0;
  for (int i = 0; i < batch; ++i) {
    const pfm_band_problem &P = probs[i];
    BandDesc &D = desc[i];
    memset(&D, 0, sizeof D);
    D.bands = P.bands;
    D.V = P.V;
    D.Fe = P.F_exp;
    D.Fp = P.F_phi1;
    D.ldv = P.ldv;
    D.ldf = P.ldf;
    D.d = P.d;
    D.p = P.p;
    D.b = b;
    D.theta = theta;
    const int64_t d = P.d, p = P.p;
    D.b_off = dofs; dofs += align_up((2 * b + 1) * d, 64);
    D.f_off = dofs; dofs += align_up((int64_t)T.nterms * (2 * b + 1) * d, 64);
    D.wave0 = (int32_t)waves;
    D.sg0 = (int32_t)sgs;
    if (b == 2 && T.nterms <= 8 && d <= kTsMaxD) {
      // band_scan_kernel: the vector stays on chip, no vectors or checkpoints
      D.nsg = T.nf * (int32_t)((p + kBsC - 1) / kBsC);
      sgs += D.nsg;
    } else {
      D.v_off = dofs; dofs += align_up((int64_t)T.nf * 3 * d * p, 64);
      D.z_off = dofs; dofs += align_up((int64_t)T.nf * ((d + kBandL(b) - 1) / kBandL(b)) * T.nterms * b * p, 64);
      D.nwaves = T.nf * (int32_t)((p + 63) / 64);
      waves += D.nwaves;
    }
    if (waves > (int64_t)1 << 30 || sgs > (int64_t)1 << 30)
      return set_err(ctx, PFM_ERR_INVALID, "too many columns in one call");
  }
  const int64_t desc_bytes = align_up((int64_t)batch * sizeof(BandDesc), 256);
  const int64_t plan_bytes = align_up((int64_t)batch * sizeof(PlanRec), 256);
  rc = ws_reserve(ctx, desc_bytes + plan_bytes + dofs * 8, stream);
  if (rc) return rc;
  char *base = (char *)ctx->ws;
  BandDesc *d_desc = (BandDesc *)base;
  PlanRec *d_plan = (PlanRec *)(base + desc_bytes);
  double *wsd = (double *)(base + desc_bytes + plan_bytes);
  rc = upload_desc(ctx, d_desc, desc.data(), batch * sizeof(BandDesc), stream);
  if (rc) return rc;
  hipLaunchKernelGGL(band_plan_kernel, dim3(batch), dim3(256), 0, stream, d_desc, d_plan, force_plan);
  HIP_TRY(ctx, hipGetLastError());
  {
    int rcp = prof_harvest(ctx);
    if (rcp) return rcp;
  }
  // phase timing (pfm_profile): 0 the factorisations, 1 the N steps
  for (int ph = 0; ph < kNumPhases; ++ph) ctx->cur_launches[ph] = 0;
  prof_mark(ctx, 0, stream);
  const int nfac = batch * T.nterms;
  {
    const dim3 gf((nfac + 63) / 64);
    if (b == 1) hipLaunchKernelGGL(band_factor_kernel<1>, gf, dim3(64), 0, stream, d_desc, d_plan, batch, T, wsd);
    else if (b == 2) hipLaunchKernelGGL(band_factor_kernel<2>, gf, dim3(64), 0, stream, d_desc, d_plan, batch, T, wsd);
    else if (b == 3) hipLaunchKernelGGL(band_factor_kernel<3>, gf, dim3(64), 0, stream, d_desc, d_plan, batch, T, wsd);
    else hipLaunchKernelGGL(band_factor_kernel<4>, gf, dim3(64), 0, stream, d_desc, d_plan, batch, T, wsd);
  }
  ctx->cur_launches[0]++;
  prof_mark(ctx, 1, stream);
  if (sgs) {
    const bool band_phi = T.fn[0] == 1 || (T.nf > 1 && T.fn[1] == 1);
    const dim3 gs((unsigned)align_up(sgs, 8));
#define PFM_BAND_SCAN(NT)                                                                                        \
  do {                                                                                                           \
    if (band_phi)                                                                                                \
      hipLaunchKernelGGL((band_scan_kernel<NT, true>), gs, dim3(64 * NT), 0, stream, d_desc, batch, d_plan, T,   \
                         (const double *)wsd, (int)sgs);                                                         \
    else                                                                                                         \
      hipLaunchKernelGGL((band_scan_kernel<NT, false>), gs, dim3(64 * NT), 0, stream, d_desc, batch, d_plan, T,  \
                         (const double *)wsd, (int)sgs);                                                         \
  } while (0)
    if (T.nterms == 4) PFM_BAND_SCAN(4);
    else if (T.nterms == 5) PFM_BAND_SCAN(5);
    else PFM_BAND_SCAN(8);
#undef PFM_BAND_SCAN
  }
#define PFM_BAND_STEPS(BW, NT)                                                                                 \
  if (waves)                                                                                                   \
  hipLaunchKernelGGL((band_steps_kernel<BW, NT>), dim3((unsigned)waves), dim3(64), 0, stream, d_desc, batch, d_plan, \
                     T, (const double *)wsd, wsd)
#define PFM_BAND_NT(BW)                                   \
  switch (T.nterms) {                                     \
    case 4: PFM_BAND_STEPS(BW, 4); break;                 \
    case 5: PFM_BAND_STEPS(BW, 5); break;                 \
    case 8: PFM_BAND_STEPS(BW, 8); break;                 \
    default: PFM_BAND_STEPS(BW, 10); break;               \
  }
  switch (b) {
    case 1: PFM_BAND_NT(1); break;
    case 2: PFM_BAND_NT(2); break;
    case 3: PFM_BAND_NT(3); break;
    default: PFM_BAND_NT(4); break;
  }
#undef PFM_BAND_NT
#undef PFM_BAND_STEPS
  ctx->cur_launches[1]++;
  prof_mark(ctx, 2, stream);
  prof_mark(ctx, 3, stream);
  if (info)
    hipLaunchKernelGGL(band_info_kernel, dim3((batch + 255) / 256), dim3(256), 0, stream, d_desc, d_plan,
                       (InfoRec *)info, batch, order);
  prof_mark(ctx, 4, stream);
  if (ctx->prof) ctx->prof_pending = true;
  HIP_TRY(ctx, hipGetLastError());
  return PFM_OK;
}

int pfm_check(pfm_ctx *ctx, pfm_stream_t stream) {
  if (!ctx) return PFM_ERR_INVALID;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize((hipStream_t)stream));
  int flags[16];
  HIP_TRY(ctx, hipMemcpy(flags, ctx->d_err, sizeof flags, hipMemcpyDeviceToHost));
  if (flags[0]) {
    HIP_TRY(ctx, hipMemset(ctx->d_err, 0, 64));
    return set_err(ctx, PFM_ERR_DEVICE, "device-side wait timed out or scheduler overflow (flags 0x%x)",
                   flags[0]);
  }
  return PFM_OK;
}

// Test hook: run one FP64 MFMA on known operands and copy the 64 x 4
// accumulator values to host memory `out`.
int pfm_selftest_mfma(int device, double *out) {
  if (!out) return PFM_ERR_INVALID;
  if (hipSetDevice(device) != hipSuccess) return PFM_ERR_HIP;
  double *d = nullptr;
  if (hipMalloc(&d, 512 * sizeof(double)) != hipSuccess) return PFM_ERR_HIP;
  hipLaunchKernelGGL(selftest_mfma_kernel, dim3(1), dim3(64), 0, 0, d);
  hipLaunchKernelGGL(selftest_mfma32_kernel, dim3(1), dim3(64), 0, 0, d + 256);
  hipError_t e = hipMemcpy(out, d, 512 * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? PFM_OK : PFM_ERR_HIP;
}

int pfm_eval_batched(pfm_ctx *ctx, int f, int m, double tol, int prec, int dtype, int batch,
                     const pfm_problem *probs, pfm_info *info, int force_plan, pfm_stream_t stream) {
  return pfm_eval_batched_tols(ctx, f, m, nullptr, tol, prec, dtype, batch, probs, info, force_plan, stream);
}

}  // extern "C"

namespace {

// A caller-given partial-fraction set (pfm_eval_rational): the terms as the
// kernels take them, and whether any shift is complex.
struct CustomSet {
  Terms T;
  bool complex_shift;
};

int eval_impl(pfm_ctx *ctx, int f, int m, const double *tols, double tol, int prec, int dtype, int batch,
              const pfm_problem *probs, pfm_info *info, int force_plan, pfm_stream_t stream_,
              const CustomSet *cs) {
  if (!ctx) return PFM_ERR_INVALID;
  const bool log1m = f == PFM_LOG1M;
  // a caller-given set: no scaling identity, r(A) itself (s = 0) or one step
  // of the action (N = 1)
  if (!valid_mask(f)) return set_err(ctx, PFM_ERR_INVALID, "bad function mask %d", f);
  const bool phi2 = !log1m && (f & PFM_PHI2);
  if (tols) {  // per-instance tolerances: the scalar is their minimum
    if (batch < 1) return set_err(ctx, PFM_ERR_INVALID, "empty batch");
    tol = tols[0];
    for (int i = 0; i < batch; ++i) {
      if (!(tols[i] > 0.0 && tols[i] < 1.0)) return set_err(ctx, PFM_ERR_INVALID, "tol must lie in (0,1)");
      tol = std::min(tol, tols[i]);
    }
  }
  if (!(tol > 0.0 && tol < 1.0)) return set_err(ctx, PFM_ERR_INVALID, "tol must lie in (0,1)");
  if (batch < 1 || !probs) return set_err(ctx, PFM_ERR_INVALID, "empty batch");
  if (prec != PFM_FP64 && prec != PFM_MIXED) return set_err(ctx, PFM_ERR_INVALID, "bad prec");
  if (dtype != PFM_R64 && dtype != PFM_C128) return set_err(ctx, PFM_ERR_INVALID, "bad dtype");
  hipStream_t stream = (hipStream_t)stream_;
  const bool action = probs[0].p > 0;
  for (int i = 0; i < batch; ++i) {
    const pfm_problem &P = probs[i];
    if (P.n < 1 || P.p < 0 || !P.A) return set_err(ctx, PFM_ERR_INVALID, "problem %d: bad n/p/A", i);
    if ((P.p > 0) != action) return set_err(ctx, PFM_ERR_INVALID, "mixed full/action batch");
    if (P.lda < P.n) return set_err(ctx, PFM_ERR_INVALID, "problem %d: lda < n", i);
    const int64_t ocols = action ? P.p : P.n;
    if (P.ldf < ocols) return set_err(ctx, PFM_ERR_INVALID, "problem %d: ldf too small", i);
    if (((f & PFM_EXP) || log1m) && !P.F_exp) return set_err(ctx, PFM_ERR_INVALID, "problem %d: F_exp null", i);
    if ((f & PFM_PHI1) && !log1m && !P.F_phi1) return set_err(ctx, PFM_ERR_INVALID, "problem %d: F_phi1 null", i);
    if (phi2 && !P.F_phi2) return set_err(ctx, PFM_ERR_INVALID, "problem %d: F_phi2 null", i);
    if (action && (!P.V || P.ldv < P.p)) return set_err(ctx, PFM_ERR_INVALID, "problem %d: bad V", i);
    if (misaligned(P.A) || misaligned(P.V) || misaligned(P.F_exp) || misaligned(P.F_phi1) ||
        (phi2 && misaligned(P.F_phi2)))
      return set_err(ctx, PFM_ERR_INVALID, "problem %d: an array is not 8-byte aligned", i);
  }
  const PfmSetEntry *ee = nullptr, *ep = nullptr;
  bool hybrid = false, pairs = false;
  if (cs) {
    if (prec != PFM_FP64)
      return set_err(ctx, PFM_ERR_UNSUPPORTED, "a caller-given set is evaluated in binary64 only");
    pairs = cs->complex_shift;  // complex shifts: the embedded route
  } else {
    ee = find_set(m, log1m ? 2 : 0);
    ep = find_set(m, 1);
    if (log1m) {
      // log(1 - A): its own set, evaluated at s = 0 (no scaling identity)
      if (!ee) return set_err(ctx, PFM_ERR_UNSUPPORTED, "no log(1 - x) set for m = %d", m);
      if (prec != PFM_FP64 || dtype != PFM_R64 || action)
        return set_err(ctx, PFM_ERR_UNSUPPORTED, "log(1 - A) is provided for real full matrices in binary64");
      ep = ee;  // the phi1 slot is never read (want_phi = 0)
    }
    hybrid = ee && (ee->poly[0] != 0.0 || ee->poly[1] != 0.0);
    if (!ee || (!ep && !hybrid)) return set_err(ctx, PFM_ERR_UNSUPPORTED, "no coefficient set for m = %d", m);
    if (hybrid) {
      // the hybrid set of §4.3: the exponential of real matrices in binary64;
      // full matrices on the Gauss-Jordan routes (checked after the plan),
      // the action on every route
      if (f != PFM_EXP || prec != PFM_FP64 || dtype != PFM_R64)
        return set_err(ctx, PFM_ERR_UNSUPPORTED,
                       "m = %d (the hybrid set) is provided for exp(A) of real matrices in binary64", m);
      ep = ee;  // no phi1 weights; never read (want_phi = 0)
    }
    pairs = ee->pair != 0;
  }
  const bool cplx = dtype == PFM_C128;
  const int order_v = cs ? 0 : ee->order;
  const bool mixed = prec == PFM_MIXED;
  const PfmSetEntry *eq = nullptr;
  if (phi2) {
    // phi2 with the squaring recurrence: real full matrices in binary64 on
    // the single-workgroup routes, real shift sets
    eq = cs ? nullptr : find_set(m, 3);
    bool small = true;
    for (int i = 0; i < batch; ++i) small &= probs[i].n <= 512;
    if (!eq || hybrid || pairs || mixed || cplx || action || !small)
      return set_err(ctx, PFM_ERR_UNSUPPORTED,
                     "phi2 is provided for real full matrices up to n = 512 in binary64 with m = 4, 5 or 8");
  }
  if (mixed && (cplx || pairs || action))
    return set_err(ctx, PFM_ERR_UNSUPPORTED,
                   "the mixed path is built for real full-matrix problems with real shift sets");
  const bool emb = cplx || pairs;  // complex arithmetic runs on the real embedding
  for (int i = 0; i < batch; ++i) {
    const int nk = emb ? 2 * probs[i].n : probs[i].n;
    if (nk <= 512) continue;
    // large instances: Gauss-Jordan route only (real shift sets, binary64)
    if (mixed || pairs)
      return set_err(ctx, PFM_ERR_UNSUPPORTED,
                     "problem %d: n = %d needs the large-instance route, which has no %s", i, probs[i].n,
                     mixed ? "mixed-precision variant" : "conjugate-pair (complex shift) variant");
    if (nk > kLargeMax)
      return set_err(ctx, PFM_ERR_UNSUPPORTED, "problem %d: n = %d exceeds the largest size (%s%d)", i,
                     probs[i].n, emb ? "complex: n <= " : "n <= ", emb ? kLargeMax / 2 : kLargeMax);
    if (action && probs[i].p > 64)
      return set_err(ctx, PFM_ERR_UNSUPPORTED, "problem %d: p = %d > 64 at n > 512 (split V)", i, probs[i].p);
  }

  double theta = INFINITY;  // a caller-given set has no bound: the caller scales A
  if (!cs) {
    const int rc = pfm_theta(f, m, tol, &theta);
    if (rc) return set_err(ctx, rc, "theta failed");
  }
  std::vector<double> thetas(batch, theta);
  if (tols && !cs) {
    std::map<double, double> seen;
    for (int i = 0; i < batch; ++i) {
      auto it = seen.find(tols[i]);
      if (it == seen.end()) {
        double th;
        if (pfm_theta(f, m, tols[i], &th)) return set_err(ctx, PFM_ERR_INVALID, "theta failed");
        it = seen.emplace(tols[i], th).first;
      }
      thetas[i] = it->second;
    }
  }
  for (int i = 0; i < (cs ? 0 : tols ? batch : 1); ++i) {
    const double ti = tols ? tols[i] : tol, th = thetas[i];
    const double fl = std::max({rounding_floor(ee, th), T_want_phi(f) ? rounding_floor(ep, th) : 0.0,
                                phi2 ? rounding_floor(eq, th) : 0.0});
    if (ti < fl)
      return set_err(ctx, PFM_ERR_UNSUPPORTED, "tol %g is below the rounding floor %.2g of the m = %d set", ti, fl, m);
  }

  Terms T;
  memset(&T, 0, sizeof T);
  if (cs) {
    T = cs->T;
  } else {
  T.want_exp = ((f & PFM_EXP) || log1m) ? 1 : 0;  // log(1 - A) runs in the exp slot
  T.want_phi = ((f & PFM_PHI1) && !log1m) || phi2 ? 1 : 0;  // phi2's doubling squares phi1
  T.want_phi2 = phi2 ? 1 : 0;
  T.a0e = ee->a0;
  T.a0p = ep->a0;
  T.a0q = phi2 ? eq->a0 : 0.0;
  T.d1e = ee->poly[0];
  T.d2e = ee->poly[1];
  if (!pairs) {
    // one real shift set shared by both functions (§2)
    T.nterms = ee->nterms;
    for (int k = 0; k < ee->nterms; ++k) {
      T.c_re[k] = ee->c_re[k];
      T.we_re[k] = ee->w_re[k];
      T.wp_re[k] = ep->w_re[k];
      T.wq_re[k] = phi2 ? eq->w_re[k] : 0.0;
    }
  } else {
    // one conjugate pair per function (the Padé poles of exp and phi1
    // differ); the exponential's pair is always needed (squaring/recurrence)
    int k = 0;
    for (int fn = 0; fn < 1 + T.want_phi; ++fn) {
      const PfmSetEntry *e = fn ? ep : ee;
      for (int cj = 0; cj < (cplx ? 2 : 1); ++cj) {  // complex A: both members
        const double sg = cj ? -1.0 : 1.0;
        T.c_re[k] = e->c_re[0];
        T.c_im[k] = sg * e->c_im[0];
        if (fn) { T.wp_re[k] = e->w_re[0]; T.wp_im[k] = sg * e->w_im[0]; }
        else { T.we_re[k] = e->w_re[0]; T.we_im[k] = sg * e->w_im[0]; }
        T.fold[k] = 1;
        T.fn[k] = fn;
        ++k;
      }
    }
    T.nterms = k;
    T.pair_real = cplx ? 0 : 1;
  }
  }
  const int nterms = T.nterms;

  // route policy: the context's, unless a tuned one exists for this batch
  int pol_gj = ctx->gj, pol_ln = ctx->ln_min, pol_direct = ctx->sq_direct, pol_t128 = kTile128Min[0];
  int pol_gjb = kGjBlock[0];
  {
    const int pidx = ctx->force_policy >= 0 ? ctx->force_policy
                                            : [&] {
                                                auto it = ctx->tuned.find(batch_key(action, emb, mixed, batch, probs));
                                                return it == ctx->tuned.end() ? -1 : it->second;
                                              }();
    if (pidx >= 0) {
      if (ctx->gj && !hybrid) {  // an explicit PFM_ROUTE_LU stays authoritative
        pol_gj = kPolicies[pidx % kNumRoutePolicies].gj;
        pol_ln = kPolicies[pidx % kNumRoutePolicies].ln_min;
      }
      if (!ctx->sched_explicit) pol_direct = kSqDirect[(pidx / kNumRoutePolicies) % kNumSchedules];
      pol_t128 = kTile128Min[(pidx / (kNumRoutePolicies * kNumSchedules)) % kNumTiles];
      pol_gjb = kGjBlock[pidx / (kNumRoutePolicies * kNumSchedules * kNumTiles)];
    }
  }
  const bool gj_call = pol_gj && !action && !emb && !mixed;
  if (hybrid && !gj_call && !action)
    for (int i = 0; i < batch; ++i)
      if (probs[i].n <= 512)
        return set_err(ctx, PFM_ERR_UNSUPPORTED,
                       "m = %d needs the Gauss-Jordan routes, which PFM_ROUTE_LU turns off (instance %d)", m, i);
  // workspace layout: from the sizes alone (the device routes each instance
  // after its plan, so every route an instance may take is laid out)
  std::vector<InstDesc> desc(batch);
  std::vector<int> cls_list[4];
  int64_t dofs = 0, iofs = 0;
  for (int i = 0; i < batch; ++i) {
    const pfm_problem &P = probs[i];
    InstDesc &D = desc[i];
    memset(&D, 0, sizeof D);
    D.Ain = (const double *)P.A;
    D.ldin = P.lda;
    D.cin = cplx ? 1 : 0;
    D.V = (const double *)P.V;
    D.Fe = (double *)P.F_exp;
    D.Fp = (double *)P.F_phi1;
    D.Fq = (double *)P.F_phi2;
    D.ldv = P.ldv;
    D.ldf = P.ldf;
    D.emb = emb ? 1 : 0;
    D.theta = thetas[i];
    D.hn = P.n;
    D.n = emb ? 2 * P.n : P.n;
    D.ncol = P.n;
    // Routes: real FP64 full-matrix instances may take the single-workgroup
    // Gauss-Jordan path (64-wide blocks); instances above 512 must take the
    // multi-workgroup one (class 3); action and complex instances above the
    // threshold take it when the shifted matrices are dominant and keep the
    // pivoting LU route otherwise, so both workspaces are laid out for them.
    const bool large = D.n > 512;
    const bool may_ln = large || (!mixed && !pairs && D.n > pol_ln && (action || emb));
    D.npad = (gj_call || may_ln) ? (D.n + 63) / 64 * 64 : (D.n + 15) / 16 * 16;
    D.rflags = (may_ln ? kRfMayLn : 0) | (large ? kRfLarge : 0) | (gj_call && !large ? kRfGj : 0);
    D.p = P.p;
    D.cls = large ? 3 : (D.npad <= 128 ? 0 : (D.npad <= 256 ? 1 : 2));
    const int64_t np = D.npad, nn = np * np;
    D.fac_off = dofs;  dofs += align_up(nterms * nn, 64);
    if (may_ln) {
      D.ln_off = dofs; dofs += align_up(nterms * ln_stride(D.npad), 64);
      if (action) {
        D.v_off = dofs;
        dofs += align_up(2 * ln_vchain(D.npad, D.p) + (int64_t)ln_ks(D.n) * np * ln_pp(D.p), 64);
      }
    }
    if (!large) {
      D.dinv_off = dofs; dofs += align_up(nterms * 2 * (np / 16) * 256, 64);
    }
    D.r_off = dofs;    dofs += align_up((phi2 ? 6 : 4) * nn, 64);
    if (emb || mixed) {
      D.e_off = dofs;  dofs += align_up((int64_t)std::max(D.n, D.npad) * D.npad, 64);
    }
    if (emb) {
      D.lda = D.n;     // A is set once the workspace base is known
    } else {
      D.A = (const double *)P.A;
      D.lda = P.lda;
    }
    if (!large) {
      D.perm_ioff = iofs; iofs += align_up(nterms * np, 64);
      D.ipiv_ioff = iofs; iofs += align_up(nterms * np, 64);
    }
    cls_list[D.cls].push_back(i);
  }
  // class 1: the npad = 256 instances first, so that the 128-block kernel
  // takes a prefix of the list and the 64-block one the rest
  int n_wide = 0;
  if (gj_call && pol_gjb == 128) {
    std::stable_partition(cls_list[1].begin(), cls_list[1].end(), [&](int i) { return desc[i].npad == 256; });
    for (int i : cls_list[1]) n_wide += desc[i].npad == 256;
  }

  // Instance lists (all from the sizes): per class for the single-workgroup
  // kernels; the multi-workgroup candidates by class; their action step
  // groups; the squaring groups by tile edge.  Kernels skip the instances the
  // device routed elsewhere.
  std::vector<int> lists;
  int cls_off[3];
  for (int c = 0; c < 3; ++c) {
    cls_off[c] = (int)lists.size();
    lists.insert(lists.end(), cls_list[c].begin(), cls_list[c].end());
  }
  std::vector<int> ln_list;
  for (int c = 0; c < 4; ++c)
    for (int i : cls_list[c])
      if (desc[i].rflags & kRfMayLn) ln_list.push_back(i);
  int ln_cls_off[5] = {0, 0, 0, 0, 0};
  for (int i : ln_list) ln_cls_off[desc[i].cls + 1]++;
  for (int c = 0; c < 4; ++c) ln_cls_off[c + 1] += ln_cls_off[c];
  const int ln_off_l = (int)lists.size();
  lists.insert(lists.end(), ln_list.begin(), ln_list.end());
  std::vector<int> act_list[4];
  int act_off[4] = {0, 0, 0, 0};
  if (action) {
    for (int i : ln_list) {
      const int np_i = desc[i].npad;
      act_list[np_i <= 256 ? 0 : np_i <= 512 ? 1 : 3].push_back(i);
    }
    for (int c = 0; c < 4; ++c) {
      act_off[c] = (int)lists.size();
      lists.insert(lists.end(), act_list[c].begin(), act_list[c].end());
    }
  }
  auto tile_of = [&](int i) { return desc[i].npad >= pol_t128 || desc[i].cls == 3 ? 1 : 0; };
  std::vector<int> sq_group[2];
  int sq_off[2] = {0, 0};
  if (!action) {
    for (int i = 0; i < batch; ++i) sq_group[tile_of(i)].push_back(i);
    for (int g = 0; g < 2; ++g) {
      sq_off[g] = (int)lists.size();
      lists.insert(lists.end(), sq_group[g].begin(), sq_group[g].end());
    }
  }
  std::vector<int> gj_cand;  // instances that may take a Gauss-Jordan route
  for (int i = 0; i < batch; ++i)
    if (desc[i].rflags & (kRfGj | kRfMayLn)) gj_cand.push_back(i);
  const bool any_gj = !gj_cand.empty();

  // GEMM task lists: level 0 = R = a0 I + S B of the Gauss-Jordan
  // candidates, the B T products of the multi-workgroup candidates, and one
  // list of every instance's tiles that each directly launched squaring level
  // reuses; per list one part per tile size (128 for npad >= 256, else 64).
  // All tiles of one instance go to one XCD.
  std::vector<SqTask> all;
  const int nchains = 1 + T.want_phi + T.want_phi2;  // products per output tile and level: R, Phi, Phi2
  using LevelLists = std::array<std::pair<int64_t, int>, 2>;  // (offset, count) per tile size
  auto build = [&](const std::vector<int> &ids, int tc, bool all_cols) {
    std::vector<std::vector<SqTask>> qx(8);
    int x = 0;
    const int TL = tc ? 128 : 64;
    for (int i : ids) {
      if (tile_of(i) != tc) continue;
      const int tlm = (desc[i].npad + TL - 1) / TL;
      const int tln = ((all_cols ? desc[i].npad : desc[i].ncol) + TL - 1) / TL;
      for (int w = 0; w < nchains; ++w)
        for (int tt = 0; tt < tlm * tln; ++tt) qx[x].push_back(SqTask{i, tt + (w << 20)});
      x = (x + 1) & 7;
    }
    size_t mx = 0;
    for (auto &q : qx) mx = std::max(mx, q.size());
    const int64_t off = (int64_t)all.size();
    for (size_t qq = 0; qq < mx; ++qq)
      for (int xx = 0; xx < 8; ++xx) all.push_back(qq < qx[xx].size() ? qx[xx][qq] : SqTask{-1, 0});
    return std::make_pair(off, (int)(mx * 8));
  };
  const LevelLists lv0{build(gj_cand, 0, false), build(gj_cand, 1, false)};
  const LevelLists lvbt{build(ln_list, 0, true), build(ln_list, 1, true)};
  std::vector<int> every(batch);
  for (int i = 0; i < batch; ++i) every[i] = i;
  LevelLists lvsq{std::make_pair((int64_t)0, 0), std::make_pair((int64_t)0, 0)};
  if (!action) lvsq = LevelLists{build(every, 0, false), build(every, 1, false)};
  // alpha1 = sum_k w_k of the binary64 weights, summed in extended precision
  double a1e = 0.0, a1p = 0.0;
  {
    long double se = 0.0L, sp = 0.0L;
    for (int k = 0; k < nterms; ++k) { se += (long double)T.we_re[k]; sp += (long double)T.wp_re[k]; }
    a1e = (double)se + T.d1e;  // the hybrid set's d1 B joins alpha1 B
    a1p = (double)sp;
  }

  // workspace tail: plans, descriptors, lists, the squaring queues
  const int64_t plan_bytes = align_up((int64_t)batch * sizeof(PlanRec), 256);
  const int64_t desc_bytes = align_up((int64_t)batch * sizeof(InstDesc), 256);
  const int64_t list_bytes = align_up((int64_t)std::max<size_t>(lists.size(), 1) * sizeof(int), 256);
  auto queue_bytes = [&](int ng) {
    return align_up(sizeof(SqQueue), 64) + align_up((int64_t)ng * 4, 64) + align_up((int64_t)(ng + 1) * 8, 64) +
           align_up((int64_t)(kSCap + 2) * 8, 64) + align_up((int64_t)ng * 4, 64);
  };
  const int64_t q_bytes = align_up(queue_bytes((int)sq_group[0].size()), 256) +
                          align_up(queue_bytes((int)sq_group[1].size()), 256);
  const int64_t need = dofs * 8 + align_up(iofs * 4, 256) + plan_bytes + desc_bytes + list_bytes + q_bytes + 4096;
  if (ctx->budget && (size_t)need > ctx->budget)
    return set_err(ctx, PFM_ERR_BUDGET, "workspace %lld bytes exceeds budget %zu", (long long)need,
                   ctx->budget);
  const size_t tb = all.size() * sizeof(SqTask);

  // a call recorded into the caller's stream capture: nothing may allocate,
  // synchronise or read host memory that a later call may change
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (stream) HIP_TRY(ctx, hipStreamIsCapturing(stream, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (capturing && ((size_t)need > ctx->ws_bytes || tb > ctx->tasks_bytes || ctx->prof))
    return set_err(ctx, PFM_ERR_INVALID,
                   "a captured call must not grow the workspace or time phases: run the same call eagerly once "
                   "first, with pfm_profile off");

  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if ((size_t)need > ctx->ws_bytes) {
    if (ctx->ws) {
      HIP_TRY(ctx, hipStreamSynchronize(stream));
      HIP_TRY(ctx, hipFree(ctx->ws));
      ctx->ws = nullptr;
      ctx->ws_bytes = 0;
    }
    ctx->up_valid = false;
    HIP_TRY(ctx, hipMalloc(&ctx->ws, (size_t)need));
    ctx->ws_bytes = (size_t)need;
  }
  if (tb > ctx->tasks_bytes) {
    if (ctx->tasks) {
      HIP_TRY(ctx, hipStreamSynchronize(stream));
      HIP_TRY(ctx, hipFree(ctx->tasks));
    }
    ctx->tasks = nullptr;
    ctx->tasks_bytes = 0;
    ctx->up_valid = false;
    HIP_TRY(ctx, hipMalloc(&ctx->tasks, std::max<size_t>(tb, 256)));
    ctx->tasks_bytes = std::max<size_t>(tb, 256);
  }
  char *base = (char *)ctx->ws;
  double *wsd = (double *)base;
  int *wsi = (int *)(base + dofs * 8);
  char *tail = base + dofs * 8 + align_up(iofs * 4, 256);
  PlanRec *d_plan = (PlanRec *)tail;
  ctx->fac_desc = desc;
  ctx->fac_nterms = nterms;
  ctx->fac_mixed = mixed;
  ctx->fac_wsd = wsd;
  ctx->fac_wsi = wsi;
  ctx->fac_plan = d_plan;
  InstDesc *d_desc = (InstDesc *)(tail + plan_bytes);
  int *d_list = (int *)(tail + plan_bytes + desc_bytes);
  char *qbase = tail + plan_bytes + desc_bytes + list_bytes;
  struct QPtr {
    SqQueue *q;
    int *ord;
    long long *pre, *lstart;
    int *done;
  } qp[2];
  {
    char *c = qbase;
    for (int g = 0; g < 2; ++g) {
      const int ng = (int)sq_group[g].size();
      char *c0 = c;
      qp[g].q = (SqQueue *)c;  c += align_up(sizeof(SqQueue), 64);
      qp[g].ord = (int *)c;    c += align_up((int64_t)ng * 4, 64);
      qp[g].pre = (long long *)c; c += align_up((int64_t)(ng + 1) * 8, 64);
      qp[g].lstart = (long long *)c; c += align_up((int64_t)(kSCap + 2) * 8, 64);
      qp[g].done = (int *)c;
      c = c0 + align_up(queue_bytes(ng), 256);
    }
  }
  for (int i = 0; i < batch; ++i)
    if (desc[i].emb) desc[i].A = wsd + desc[i].e_off;

  // descriptors, lists and task lists: uploaded through the pinned staging
  // area unless the device already holds exactly these bytes at these
  // addresses (then a captured call has no copy node at all)
  {
    const size_t nd = batch * sizeof(InstDesc), nl = lists.size() * sizeof(int);
    std::vector<char> key(nd + nl + tb + 4 * sizeof(void *));
    char *kp = key.data();
    const void *ptrs[4] = {ctx->ws, ctx->tasks, d_desc, d_list};
    memcpy(kp, ptrs, sizeof ptrs);
    memcpy(kp + sizeof ptrs, desc.data(), nd);
    memcpy(kp + sizeof ptrs + nd, lists.data(), nl);
    if (tb) memcpy(kp + sizeof ptrs + nd + nl, all.data(), tb);
    if (!(ctx->up_valid && ctx->up_key == key)) {
      if (capturing)
        return set_err(ctx, PFM_ERR_INVALID,
                       "a captured call must repeat the previous call on this context (same problems and "
                       "arguments): run it eagerly once first");
      const size_t a_nd = align_up(nd, 256), a_nl = align_up(nl, 256);
      char *pin = nullptr;
      const int rcs = staging(ctx, a_nd + a_nl + tb + 256, &pin);
      if (rcs) return rcs;
      memcpy(pin, desc.data(), nd);
      if (nl) memcpy(pin + a_nd, lists.data(), nl);
      if (tb) memcpy(pin + a_nd + a_nl, all.data(), tb);
      ctx->up_valid = false;
      HIP_TRY(ctx, hipMemcpyAsync(d_desc, pin, nd, hipMemcpyHostToDevice, stream));
      if (nl) HIP_TRY(ctx, hipMemcpyAsync(d_list, pin + a_nd, nl, hipMemcpyHostToDevice, stream));
      if (tb) HIP_TRY(ctx, hipMemcpyAsync(ctx->tasks, pin + a_nd + a_nl, tb, hipMemcpyHostToDevice, stream));
      HIP_TRY(ctx, hipEventRecord(ctx->pin_ev, stream));
      ctx->pin_pending = true;
      ctx->up_key.swap(key);
      ctx->up_valid = true;
    }
  }
  if (!capturing) {
    const int rcp = prof_harvest(ctx);
    if (rcp) return rcp;
  }
  const SqTask *dt = (const SqTask *)ctx->tasks;
  int ln_npm = 0, ln_big_npm = 0;
  for (int i : ln_list) {
    ln_npm = std::max(ln_npm, desc[i].npad);
    if (desc[i].cls == 3) ln_big_npm = std::max(ln_big_npm, desc[i].npad);
  }
  double cmax = 0.0;
  for (int k = 0; k < nterms; ++k) cmax = std::max(cmax, std::hypot(T.c_re[k], T.c_im[k]));
  int maxc = 0, maxn = 0, maxp = 0;
  for (int i = 0; i < batch; ++i) {
    maxc = std::max(maxc, probs[i].n);
    maxn = std::max(maxn, desc[i].npad);
    maxp = std::max(maxp, probs[i].p);
  }
  // resident workgroups of the persistent squaring kernels (their grids)
  int occ[2] = {0, 0};
  HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], sq_persist_kernel<64>, 256, 0));
  HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], sq_persist_kernel<128>, 256, 0));
  // the large action route's steps are launched one by one: the host needs
  // their count, the one case in which a call reads the plans back
  const bool big_action = action && !act_list[3].empty();
  if (big_action && capturing)
    return set_err(ctx, PFM_ERR_UNSUPPORTED,
                   "an action on an instance above 512 (complex: 256) reads its step count back: not capturable");

  // one launch per tile size with tasks
#define PFM_SQ(MODE, LL, LEVEL)                                                                     \
  do {                                                                                              \
    if ((LL)[0].second)                                                                             \
      hipLaunchKernelGGL((square_level_f64_kernel<MODE, 64>), dim3((LL)[0].second), dim3(256), 0, stream, \
                         d_desc, dt + (LL)[0].first, (LL)[0].second, LEVEL, wsd, d_plan, T.a0e, T.a0p, a1e,  \
                         a1p, T.a0q);                                                               \
    if ((LL)[1].second)                                                                             \
      hipLaunchKernelGGL((square_level_f64_kernel<MODE, 128>), dim3((LL)[1].second), dim3(256), 0,  \
                         stream, d_desc, dt + (LL)[1].first, (LL)[1].second, LEVEL, wsd, d_plan, T.a0e,     \
                         T.a0p, a1e, a1p, T.a0q);                                                   \
  } while (0)
  // Everything from here on depends only on what the host has decided (the
  // descriptors, lists and task lists); a call that repeats all of it
  // replays a captured graph of this sequence.
  // 1. embedding, norm, plan and route, on the device
  auto enqueue_plan = [&]() -> int {
  if (emb) {
    const int te = (maxn + 31) / 32;
    hipLaunchKernelGGL(embed_kernel, dim3(te * te, batch), dim3(256), 0, stream, d_desc, wsd);
  }
  {
    const int nb = (batch + 255) / 256;
    hipLaunchKernelGGL(plan_init_kernel, dim3(nb), dim3(256), 0, stream, d_plan, batch);
    hipLaunchKernelGGL(norm_kernel, dim3((maxc + 63) / 64, batch), dim3(256), 0, stream, d_desc, d_plan);
    hipLaunchKernelGGL(plan_finish_kernel, dim3(nb), dim3(256), 0, stream, d_desc, d_plan, batch,
                       action ? 1 : 0, cs && action ? 1 : force_plan, (log1m || (cs && !action)) ? 1 : 0);
    hipLaunchKernelGGL(route_kernel, dim3(nb), dim3(256), 0, stream, d_desc, d_plan, batch, action ? 1 : 0, cmax,
                       hybrid ? 1 : 0);
  }
  return PFM_OK;
  };
  // The large action route's steps are launched one by one: the host reads
  // their count back after the plan (the one read-back of a call) and the
  // rest of the sequence depends on it.
  int big_nmax = 0;
  if (big_action) {
    const int rcp = enqueue_plan();
    if (rcp) return rcp;
    HIP_TRY(ctx, hipGetLastError());
    std::vector<PlanRec> hp(batch);
    HIP_TRY(ctx, hipMemcpyAsync(hp.data(), d_plan, batch * sizeof(PlanRec), hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    for (int i : act_list[3])
      if (on_route(hp[i], 2)) big_nmax = std::max(big_nmax, hp[i].s);
  }
  auto enqueue = [&]() -> int {
  if (!big_action) {
    const int rcp = enqueue_plan();
    if (rcp) return rcp;
  }
  for (int p = 0; p < kNumPhases; ++p) ctx->cur_launches[p] = 0;
  prof_mark(ctx, 0, stream);
  // 2. shifted factorisations: Gauss-Jordan inverses (route 1) and pivoting
  //    LU (route 0), all (instance, shift) pairs of a class per launch
  for (int c = 0; c < 3 && gj_call; ++c) {
    const int nl = (int)cls_list[c].size();
    if (!nl) continue;
    const int *dl = d_list + cls_off[c];
    const dim3 gg(xcd_grid(nl, nterms));
    if (c == 0) hipLaunchKernelGGL((gj_inv_kernel<128, false>), gg, dim3(256), 0, stream, d_desc, dl, nl, d_plan, T, wsd, 1);
    if (c == 1) {
      if (n_wide)
        hipLaunchKernelGGL((gj2_inv_kernel<false>), dim3(xcd_grid(n_wide, nterms)), dim3(512), 0, stream, d_desc, dl,
                           n_wide, d_plan, T, wsd, 1);
      if (nl > n_wide)
        hipLaunchKernelGGL((gj_inv_kernel<256, false>), dim3(xcd_grid(nl - n_wide, nterms)), dim3(256), 0, stream,
                           d_desc, dl + n_wide, nl - n_wide, d_plan, T, wsd, 1);
    }
    if (c == 2) hipLaunchKernelGGL((gj_inv_kernel<512, false>), gg, dim3(256), 0, stream, d_desc, dl, nl, d_plan, T, wsd, 1);
    ctx->cur_launches[0]++;
  }
  for (int c = 0; c < 3; ++c) {
    const int nl = (int)cls_list[c].size();
    if (!nl) continue;
    const int *dl = d_list + cls_off[c];
    const dim3 glu(xcd_grid(nl, nterms));
    const int am = action ? 1 : 0;
#define PFM_LU(NPM)                                                                            \
  do {                                                                                         \
    if (mixed)                                                                                 \
      hipLaunchKernelGGL((lu_kernel<NPM, float>), glu, dim3(256), 0, stream, d_desc, dl, nl,  \
                         d_plan, T, wsd, wsi, am);                                             \
    else                                                                                       \
      hipLaunchKernelGGL((lu_kernel<NPM, double>), glu, dim3(256), 0, stream, d_desc, dl, nl, \
                         d_plan, T, wsd, wsi, am);                                             \
  } while (0)
    if (c == 0) PFM_LU(128);
    if (c == 1) PFM_LU(256);
    if (c == 2) PFM_LU(512);
#undef PFM_LU
    ctx->cur_launches[0]++;
  }
  for (int c = 0; c < 3; ++c) {
    // multi-workgroup-route instances of a small class: one launch
    const int nl = ln_cls_off[c + 1] - ln_cls_off[c];
    if (!nl) continue;
    const int *dl = d_list + ln_off_l + ln_cls_off[c];
    const dim3 gg(xcd_grid(nl, nterms));
#define PFM_GJ_LN(NPM)                                                                             \
  do {                                                                                             \
    if (action)                                                                                    \
      hipLaunchKernelGGL((gj_inv_kernel<NPM, true>), gg, dim3(256), 0, stream, d_desc, dl, nl, d_plan, T, wsd, 2); \
    else                                                                                           \
      hipLaunchKernelGGL((gj_inv_kernel<NPM, false>), gg, dim3(256), 0, stream, d_desc, dl, nl, d_plan, T, wsd, 2); \
  } while (0)
    if (c == 0) PFM_GJ_LN(128);
    if (c == 1) PFM_GJ_LN(256);
    if (c == 2) PFM_GJ_LN(512);
#undef PFM_GJ_LN
    ctx->cur_launches[0]++;
  }
  if (ln_cls_off[4] > ln_cls_off[3]) {
    // class 3: W_k = I - c_k B, then one (pivot inverse, row, update)
    // launch triple per 64-column block step, every (instance, shift) in
    // each launch
    const int nbig = ln_cls_off[4] - ln_cls_off[3];
    const int nslot = nbig * nterms;
    const int t1 = ln_big_npm / kLB, nR = (ln_big_npm + kLRows - 1) / kLRows;
    const int *dl = d_list + ln_off_l + ln_cls_off[3];
    hipLaunchKernelGGL(ln_load_kernel, dim3(xcd_grid(nslot, t1 * t1)), dim3(256), 0, stream, d_desc, dl,
                       nslot, t1, d_plan, T, wsd, action ? 1 : 0);
    for (int J = 0; J < t1; ++J) {
      hipLaunchKernelGGL(ln_dinv_kernel, dim3(nslot), dim3(256), 0, stream, d_desc, dl, nslot, T, wsd, J, d_plan);
      hipLaunchKernelGGL(ln_row_kernel, dim3(xcd_grid(nslot, t1)), dim3(256), 0, stream, d_desc, dl, nslot,
                         t1, T, wsd, J, d_plan);
      hipLaunchKernelGGL(ln_upd_kernel, dim3(xcd_grid(nslot, t1 * nR)), dim3(256), 0, stream, d_desc, dl,
                         nslot, t1, nR, T, wsd, J, d_plan);
    }
    ctx->cur_launches[0] += 1 + 3 * t1;
  }
  prof_mark(ctx, 1, stream);
  if (action) {
    // 3'. B = A / N column-major, then the N-step recurrence per column slab
    const int tnb = (maxn + 31) / 32;
    hipLaunchKernelGGL(prep_bt_kernel, dim3(tnb * tnb, batch), dim3(256), 0, stream, d_desc, d_plan, wsd, 1);
    for (int c = 0; c < 3; ++c) {
      const int nl = (int)cls_list[c].size();
      if (!nl) continue;
      const int *dl = d_list + cls_off[c];
#define PFM_ACT(NPM, SWW)                                                                       \
  do {                                                                                          \
    const int ns = (maxp + SWW - 1) / SWW;                                                      \
    const dim3 ga(xcd_grid(nl, ns));                                                            \
    if (T.want_exp)                                                                             \
      hipLaunchKernelGGL((action_f64_kernel<NPM, SWW, false>), ga, dim3(256), 0, stream, d_desc, \
                         dl, nl, ns, d_plan, T, wsd, wsi);                                      \
    if (T.want_phi)                                                                             \
      hipLaunchKernelGGL((action_f64_kernel<NPM, SWW, true>), ga, dim3(256), 0, stream, d_desc,  \
                         dl, nl, ns, d_plan, T, wsd, wsi);                                      \
  } while (0)
      if (c == 0) PFM_ACT(128, 16);
      if (c == 1) PFM_ACT(256, 16);
      if (c == 2) PFM_ACT(512, 16);
#undef PFM_ACT
      ctx->cur_launches[1] += T.want_exp + T.want_phi;
    }
    const int nln = (int)ln_list.size();
    if (nln) {
      // large instances: S = sum_k w_k X_k, R = a0 I + S B and P (phi1),
      // then the N steps U <- R U (+ U1) as K-split GEMMs
      const int chunks = (int)(((int64_t)ln_npm * ln_npm / 4 + 255) / 256);
      const int *dl = d_list + ln_off_l;
      hipLaunchKernelGGL(combine_inv_kernel, dim3(chunks, nln), dim3(256), 0, stream, d_desc, dl, T, wsd, d_plan);
      PFM_SQ(2, lvbt, 1);  // level argument 1: B = A / N
      PFM_SQ(1, lv0, 1);
      const int nchain = T.want_exp + T.want_phi;
      for (int c = 0; c < 2; ++c) {  // one launch runs all N steps
        const int nl = (int)act_list[c].size();
        if (!nl) continue;
        int mp = 1;
        for (int i : act_list[c]) mp = std::max(mp, desc[i].p);
        const int nslab = (mp + 15) / 16;
        const int *dla = d_list + act_off[c];
        const dim3 gs(xcd_grid(nl, nchain * nslab));
        if (c == 0)
          hipLaunchKernelGGL(ln_steps_kernel<256>, gs, dim3(256), 0, stream, d_desc, dla, nl, nslab, d_plan, wsd,
                             T.want_exp, T.want_phi);
        if (c == 1)
          hipLaunchKernelGGL(ln_steps_kernel<512>, gs, dim3(256), 0, stream, d_desc, dla, nl, nslab, d_plan, wsd,
                             T.want_exp, T.want_phi);
        ctx->cur_launches[1]++;
      }
      const int nbig = (int)act_list[3].size();
      if (nbig) {
        // the large action instances, big_nmax steps (read back above)
        const int *dlb = d_list + act_off[3];
        int big_npm = 0;
        for (int i : act_list[3]) big_npm = std::max(big_npm, desc[i].npad);
        hipLaunchKernelGGL(ln_vprep_kernel, dim3(big_npm / 64, nbig), dim3(256), 0, stream, d_desc, dlb, nchain,
                           wsd, d_plan);
        int ppmask = 0, ksmax = 1;
        for (int i : act_list[3]) {
          ppmask |= 1 << (ln_pp(desc[i].p) / 16 - 1);
          ksmax = std::max(ksmax, ln_ks(desc[i].n));
        }
        const int nsub = (big_npm / 64) * ksmax;
        const dim3 gv(xcd_grid(nbig, nsub));
        for (int j = 1; j <= big_nmax; ++j) {
          for (int ch = 0; ch < nchain; ++ch) {
            const int phi = (ch == 1 || !T.want_exp) ? 1 : 0;
            const int use_p = phi && j == 1;
            const int inb = (j - 1) & 1, outb = j & 1;
#define PFM_GEMV(PPV)                                                                              \
  if (ppmask & (1 << (PPV / 16 - 1)))                                                            \
    hipLaunchKernelGGL(ln_gemv_kernel<PPV>, gv, dim3(256), 0, stream, d_desc, dlb, nbig, nsub, d_plan, \
                       wsd, j, ch, use_p, inb);
            PFM_GEMV(16) PFM_GEMV(32) PFM_GEMV(48) PFM_GEMV(64)
#undef PFM_GEMV
            hipLaunchKernelGGL(ln_vreduce_kernel, dim3(big_npm / 64, nbig), dim3(256), 0, stream, d_desc, dlb,
                               d_plan, wsd, j, ch, outb, 1.0, phi);
            ctx->cur_launches[1] += 2;
          }
        }
      }
      ctx->cur_launches[1] += 3;
    }
    prof_mark(ctx, 2, stream);
    prof_mark(ctx, 3, stream);
    prof_mark(ctx, 4, stream);
    if (ctx->prof) ctx->prof_pending = true;
    if (info)
      hipLaunchKernelGGL(info_kernel, dim3((batch + 255) / 256), dim3(256), 0, stream, d_desc, d_plan,
                         (InfoRec *)info, batch, order_v);
    HIP_TRY(ctx, hipGetLastError());
    return PFM_OK;
  }
  // 3. solves fused with the combination
  if (mixed) {
    const int tnb = (maxn + 31) / 32;
    hipLaunchKernelGGL(prep_bt_kernel, dim3(tnb * tnb, batch), dim3(256), 0, stream, d_desc, d_plan, wsd, 0);
    double sw = 0.0, swp = 0.0;
    for (int k = 0; k < nterms; ++k) { sw += std::fabs(T.we_re[k]); swp += std::fabs(T.wp_re[k]); }
    const double irtol = tol / (4.0 * std::max(sw, T.want_phi ? swp : 0.0));
    const int maxit = 3;
    for (int c = 0; c < 3; ++c) {
      const int nl = (int)cls_list[c].size();
      if (!nl) continue;
      const int *dl = d_list + cls_off[c];
#define PFM_MIX(NPM, SWW)                                                                         \
  do {                                                                                            \
    const dim3 gs(xcd_grid(nl, NPM / SWW));                                                       \
    if (T.want_phi)                                                                               \
      hipLaunchKernelGGL((solve_mixed_kernel<NPM, SWW, true>), gs, dim3(256), 0, stream, d_desc, \
                         dl, nl, d_plan, T, wsd, wsi, maxit, irtol);                              \
    else                                                                                          \
      hipLaunchKernelGGL((solve_mixed_kernel<NPM, SWW, false>), gs, dim3(256), 0, stream, d_desc,\
                         dl, nl, d_plan, T, wsd, wsi, maxit, irtol);                              \
  } while (0)
      if (c == 0) PFM_MIX(128, 16);
      if (c == 1) PFM_MIX(256, 16);
      if (c == 2) PFM_MIX(512, 16);
#undef PFM_MIX
      ctx->cur_launches[1]++;
    }
  }
  if (any_gj) {
    // S = sum_k w_k X_k, then R = a0 I + S B (and Phi) for the Gauss-Jordan instances
    int maxnp = 0;
    for (int i : gj_cand) maxnp = std::max(maxnp, desc[i].npad);
    const int chunks = (int)(((int64_t)maxnp * maxnp / 4 + 255) / 256);
    for (int c = 0; c < 3 && gj_call; ++c) {
      const int nl = (int)cls_list[c].size();
      if (!nl) continue;
      hipLaunchKernelGGL(combine_inv_kernel, dim3(chunks, nl), dim3(256), 0, stream, d_desc,
                         d_list + cls_off[c], T, wsd, d_plan);
    }
    const int nln = (int)ln_list.size();
    if (nln)
      hipLaunchKernelGGL(combine_inv_kernel, dim3(chunks, nln), dim3(256), 0, stream, d_desc,
                         d_list + ln_off_l, T, wsd, d_plan);
    PFM_SQ(2, lvbt, 0);
    PFM_SQ(1, lv0, 0);
    ctx->cur_launches[1] += 2;
  }
  for (int c = 0; c < 3 && !mixed; ++c) {
    const int nl = (int)cls_list[c].size();
    if (!nl) continue;
    const int *dl = d_list + cls_off[c];
#define PFM_SOLVE(NPM, SWW)                                                                      \
  do {                                                                                           \
    const dim3 gs(xcd_grid(nl, NPM / SWW));                                                      \
    if (T.want_phi)                                                                              \
      hipLaunchKernelGGL((solve_full_f64_kernel<NPM, SWW, true>), gs, dim3(256), 0, stream,     \
                         d_desc, dl, nl, d_plan, T, wsd, wsi);                                   \
    else                                                                                         \
      hipLaunchKernelGGL((solve_full_f64_kernel<NPM, SWW, false>), gs, dim3(256), 0, stream,    \
                         d_desc, dl, nl, d_plan, T, wsd, wsi);                                   \
  } while (0)
    if (c == 0) PFM_SOLVE(128, 32);
    if (c == 1) PFM_SOLVE(256, 16);
    if (c == 2) PFM_SOLVE(512, 16);
#undef PFM_SOLVE
    ctx->cur_launches[1]++;
  }
  prof_mark(ctx, 2, stream);
  // 4. squaring levels: the first pol_direct levels one launch each over
  //    every instance's tiles (tiles of instances with s < level return at
  //    once), the rest, whatever s is, from the persistent queue
  for (int j = 1; j <= pol_direct; ++j) {
    PFM_SQ(0, lvsq, j);
    ctx->cur_launches[2]++;
  }
  for (int g = 0; g < 2; ++g) {
    const int ng = (int)sq_group[g].size();
    if (!ng) continue;
    const int *gl = d_list + sq_off[g];
    hipLaunchKernelGGL(sq_queue_kernel, dim3(1), dim3(kQueueThreads), 0, stream, d_desc, d_plan, gl, ng,
                       g ? 128 : 64, nchains, pol_direct + 1, qp[g].q, qp[g].ord, qp[g].pre, qp[g].lstart,
                       qp[g].done);
    const int grid = std::max(1, occ[g] * ctx->num_cu);
    if (g == 0)
      hipLaunchKernelGGL(sq_persist_kernel<64>, dim3(grid), dim3(256), 0, stream, d_desc, d_plan, gl,
                         nchains, qp[g].q, qp[g].ord, qp[g].pre, qp[g].lstart, qp[g].done, wsd, ctx->d_err);
    else
      hipLaunchKernelGGL(sq_persist_kernel<128>, dim3(grid), dim3(256), 0, stream, d_desc, d_plan, gl,
                         nchains, qp[g].q, qp[g].ord, qp[g].pre, qp[g].lstart, qp[g].done, wsd, ctx->d_err);
    ctx->cur_launches[2] += 2;
  }
  prof_mark(ctx, 3, stream);
  // 5. results to the caller's row-major buffers, then the info records
  const int tn = (maxc + 31) / 32;  // stores run over the caller's n
  hipLaunchKernelGGL(store_full_kernel, dim3(tn * tn, batch), dim3(256), 0, stream, d_desc, d_plan,
                     wsd, T.want_exp, (f & PFM_PHI1) && !log1m ? 1 : 0, T.want_phi2);
  ctx->cur_launches[3]++;
  prof_mark(ctx, 4, stream);
  if (ctx->prof) ctx->prof_pending = true;
  if (info)
    hipLaunchKernelGGL(info_kernel, dim3((batch + 255) / 256), dim3(256), 0, stream, d_desc, d_plan,
                       (InfoRec *)info, batch, order_v);
  HIP_TRY(ctx, hipGetLastError());
  return PFM_OK;
  };
#undef PFM_SQ

  // hipGraph reuse: eager the first time a launch sequence is seen; captured
  // and instantiated when the same sequence comes a second time in a row;
  // replayed from then on (for a large action, the sequence after the
  // read-back, with its step count in the signature).  Not on the null
  // stream (it cannot be captured), while phase timing is on, or inside the
  // caller's own capture.
  if (!ctx->graphs || ctx->prof || stream == nullptr || capturing) return enqueue();
  uint64_t sig = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t nbytes) {  // 64-bit words, then the tail bytes
    const unsigned char *b = (const unsigned char *)p;
    size_t q = 0;
    for (; q + 8 <= nbytes; q += 8) {
      uint64_t w;
      memcpy(&w, b + q, 8);
      sig = (sig ^ w) * 1099511628211ull;
      sig ^= sig >> 29;
    }
    for (; q < nbytes; ++q) sig = (sig ^ b[q]) * 1099511628211ull;
  };
  const void *ptrs[7] = {ctx->ws, ctx->tasks, info, stream, d_desc, d_list, ctx->d_err};
  const int64_t ints[13] = {f, m, prec, dtype, batch, force_plan, pol_gj, pol_direct, pol_t128, ctx->num_cu,
                            (int64_t)lists.size(), big_nmax, pol_gjb};
  const double dbls[6] = {tol, theta, a1e, a1p, T.a0e, cmax};
  mix(ptrs, sizeof ptrs);
  mix(ints, sizeof ints);
  mix(dbls, sizeof dbls);
  mix(&T, sizeof T);
  mix(desc.data(), desc.size() * sizeof(InstDesc));
  mix(lists.data(), lists.size() * sizeof(int));
  mix(all.data(), all.size() * sizeof(SqTask));
  if (ctx->gexec && sig == ctx->gsig) {
    HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, stream));
    ++ctx->graph_replays;
    return PFM_OK;
  }
  if (sig != ctx->gseen) {  // first sighting: run eagerly, remember it
    ctx->gseen = sig;
    return enqueue();
  }
  HIP_TRY(ctx, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  const int rce = enqueue();
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(stream, &g);
  if (rce) {
    if (g) (void)hipGraphDestroy(g);
    return rce;
  }
  if (ec != hipSuccess) return set_err(ctx, PFM_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ec));
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->gexec = nullptr;
  ctx->graph = g;
  ctx->gsig = 0;
  HIP_TRY(ctx, hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
  ctx->gsig = sig;
  HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, stream));
  ++ctx->graph_captures;
  return PFM_OK;
}

}  // namespace

extern "C" {

int pfm_eval_batched_tols(pfm_ctx *ctx, int f, int m, const double *tols, double tol, int prec, int dtype,
                          int batch, const pfm_problem *probs, pfm_info *info, int force_plan,
                          pfm_stream_t stream) {
  return eval_impl(ctx, f, m, tols, tol, prec, dtype, batch, probs, info, force_plan, stream, nullptr);
}

int pfm_eval_rational(pfm_ctx *ctx, int nterms, const double *c_re, const double *c_im, const double *w_re,
                      const double *w_im, double a0, int conj_pairs, int dtype, int batch,
                      const pfm_problem *probs, pfm_info *info, pfm_stream_t stream) {
  if (!ctx) return PFM_ERR_INVALID;
  if (nterms < 1 || nterms > kMaxTerms || !c_re || !w_re)
    return set_err(ctx, PFM_ERR_INVALID, "nterms must lie in [1, %d], with c_re and w_re given", kMaxTerms);
  if (dtype != PFM_R64 && dtype != PFM_C128) return set_err(ctx, PFM_ERR_INVALID, "bad dtype");
  if (!std::isfinite(a0)) return set_err(ctx, PFM_ERR_INVALID, "a0 is not finite");
  bool any_complex = false;
  for (int k = 0; k < nterms; ++k) {
    const double ci = c_im ? c_im[k] : 0.0, wi = w_im ? w_im[k] : 0.0;
    if (!std::isfinite(c_re[k]) || !std::isfinite(ci) || !std::isfinite(w_re[k]) || !std::isfinite(wi))
      return set_err(ctx, PFM_ERR_INVALID, "term %d is not finite", k);
    if (ci == 0.0 && wi != 0.0 && dtype == PFM_R64)
      return set_err(ctx, PFM_ERR_INVALID, "term %d: a real shift with a complex weight on real A", k);
    any_complex |= ci != 0.0;
  }
  if (any_complex && dtype == PFM_R64 && !conj_pairs)
    return set_err(ctx, PFM_ERR_UNSUPPORTED,
                   "complex shifts on real A give a complex r(A): pass conj_pairs, or complex A and outputs");
  CustomSet cs;
  memset(&cs, 0, sizeof cs);
  Terms &T = cs.T;
  T.want_exp = 1;
  T.a0e = a0;
  const bool emb = any_complex || dtype == PFM_C128;
  if (!emb) {
    // real shifts and weights on real A: the real routes
    T.nterms = nterms;
    for (int k = 0; k < nterms; ++k) {
      T.c_re[k] = c_re[k];
      T.we_re[k] = w_re[k];
    }
  } else {
    // the embedded route, each weight folded into its solve's right-hand
    // side; on real A every term counts 2 Re(w_k Z_k): a complex shift for
    // itself and its conjugate, a real one with half its weight (exact)
    const bool pr = dtype == PFM_R64;
    int k2 = 0;
    auto add = [&](double cr, double ci, double wr, double wi) -> bool {
      if (k2 >= kMaxTerms) return false;
      T.c_re[k2] = cr;
      T.c_im[k2] = ci;
      T.we_re[k2] = wr;
      T.we_im[k2] = wi;
      T.fold[k2] = 1;
      T.fn[k2] = 0;
      ++k2;
      return true;
    };
    for (int k = 0; k < nterms; ++k) {
      const double ci = c_im ? c_im[k] : 0.0, wi = w_im ? w_im[k] : 0.0;
      bool ok;
      if (pr) ok = ci != 0.0 ? add(c_re[k], ci, w_re[k], wi) : add(c_re[k], 0.0, 0.5 * w_re[k], 0.0);
      else {
        ok = add(c_re[k], ci, w_re[k], wi);
        if (ok && conj_pairs && ci != 0.0) ok = add(c_re[k], -ci, w_re[k], -wi);
      }
      if (!ok) return set_err(ctx, PFM_ERR_INVALID, "more than %d solves with the conjugates", kMaxTerms);
    }
    T.nterms = k2;
    T.pair_real = pr ? 1 : 0;
  }
  cs.complex_shift = emb;
  return eval_impl(ctx, PFM_EXP, 0, nullptr, 0.5, PFM_FP64, dtype, batch, probs, info, -1, stream, &cs);
}

int pfm_set_graphs(pfm_ctx *ctx, int enable) {
  if (!ctx) return PFM_ERR_INVALID;
  ctx->graphs = enable != 0;
  return PFM_OK;
}

int pfm_graph_stats(pfm_ctx *ctx, int *captures, int *replays) {
  if (!ctx) return PFM_ERR_INVALID;
  if (captures) *captures = ctx->graph_captures;
  if (replays) *replays = ctx->graph_replays;
  return PFM_OK;
}

int pfm_tune(pfm_ctx *ctx, int f, int m, double tol, int prec, int dtype, int batch, const pfm_problem *probs,
             int reps, pfm_stream_t stream_, int *policy, double *ms) {
  if (!ctx || !probs || batch < 1 || reps < 1) return PFM_ERR_INVALID;
  const PfmSetEntry *ee = find_set(m, 0);
  if (!ee) return set_err(ctx, PFM_ERR_UNSUPPORTED, "no coefficient set for m = %d", m);
  hipStream_t stream = (hipStream_t)stream_;
  const bool action = probs[0].p > 0;
  const bool emb = dtype == PFM_C128 || ee->pair != 0;
  const bool mixed = prec == PFM_MIXED;
  // candidates that can differ for this kind of batch: the route policy
  // (full real matrices: Gauss-Jordan vs LU; action or complex: the
  // multi-workgroup route above 128 vs above 512), and for full matrices the
  // squaring schedule (levels launched one by one, or all from the
  // persistent queue) and the product tile (128 from npad 256 on, or 64)
  std::vector<int> routes = (!action && !emb) ? std::vector<int>{0, 1} : std::vector<int>{0, 2};
  // the tile choice only differs for a padded size of 256 or more
  bool tile_matters = false, block_matters = false;
  for (int i = 0; i < batch; ++i) {
    tile_matters |= (emb ? 2 * probs[i].n : probs[i].n) > 192;
    block_matters |= !action && !emb && !mixed && probs[i].n > 192 && probs[i].n <= 256;
  }
  std::vector<int> cand;
  for (int gb = 0; gb < (block_matters ? kNumGjBlocks : 1); ++gb)
    for (int tl = 0; tl < (action || !tile_matters ? 1 : kNumTiles); ++tl)
      for (int sc = 0; sc < (action ? 1 : kNumSchedules); ++sc)
        for (int r : routes) {
          if (gb && !kPolicies[r].gj) continue;  // the pivot block only matters on the Gauss-Jordan route
          cand.push_back(r + kNumRoutePolicies * (sc + kNumSchedules * (tl + kNumTiles * gb)));
        }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  const bool graphs = ctx->graphs;
  ctx->graphs = false;
  int best = -1;
  double best_ms = 0.0;
  int rc = PFM_OK;
  for (int pi : cand) {
    ctx->force_policy = pi;
    rc = pfm_eval_batched(ctx, f, m, tol, prec, dtype, batch, probs, nullptr, -1, stream);  // warm-up
    if (rc) break;
    (void)hipEventRecord(e0, stream);
    for (int r = 0; r < reps && !rc; ++r) rc = pfm_eval_batched(ctx, f, m, tol, prec, dtype, batch, probs, nullptr, -1, stream);
    (void)hipEventRecord(e1, stream);
    if (rc) break;
    (void)hipEventSynchronize(e1);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    const double per = t / reps;
    if (best < 0 || per < best_ms) {
      best = pi;
      best_ms = per;
    }
  }
  ctx->force_policy = -1;
  ctx->graphs = graphs;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  ctx->tuned[batch_key(action, emb, mixed, batch, probs)] = best;
  if (policy) *policy = best;
  if (ms) *ms = best_ms;
  return PFM_OK;
}

int pfm_tune_export(const pfm_ctx *ctx, char *buf, size_t size) {
  if (!ctx) return PFM_ERR_INVALID;
  std::string s;
  for (const auto &kv : ctx->tuned) {
    char line[64];
    snprintf(line, sizeof line, "%llu %d\n", (unsigned long long)kv.first, kv.second);
    s += line;
  }
  if (buf && size > 0) {
    const size_t k = std::min(size - 1, s.size());
    memcpy(buf, s.data(), k);
    buf[k] = 0;
  }
  return (int)s.size() + 1;
}

int pfm_lu_factors(pfm_ctx *ctx, int instance, int shift, double *lu, int64_t ldlu, int32_t *ipiv, int32_t *npad) {
  if (!ctx) return PFM_ERR_INVALID;
  if (instance < 0 || instance >= (int)ctx->fac_desc.size() || shift < 0 || shift >= ctx->fac_nterms)
    return set_err(ctx, PFM_ERR_INVALID, "pfm_lu_factors: no factorisation (%d, %d) from the last call", instance, shift);
  const InstDesc &D = ctx->fac_desc[instance];
  const int np = D.npad;
  if (npad) *npad = np;
  if (!lu && !ipiv) return PFM_OK;
  if (!lu || !ipiv || ldlu < np)
    return set_err(ctx, PFM_ERR_INVALID, "pfm_lu_factors: lu (ld >= %d) and ipiv are required", np);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipDeviceSynchronize());
  PlanRec P;
  HIP_TRY(ctx, hipMemcpy(&P, ctx->fac_plan + instance, sizeof P, hipMemcpyDeviceToHost));
  if (!on_route(P, 0))
    return set_err(ctx, PFM_ERR_INVALID, "pfm_lu_factors: instance %d did not take the pivoting LU route", instance);
  const int64_t nn = (int64_t)np * np;
  std::vector<double> w(nn);
  if (ctx->fac_mixed) {
    std::vector<float> wf(nn);
    const float *src = reinterpret_cast<const float *>(ctx->fac_wsd + D.fac_off) + (int64_t)shift * nn;
    HIP_TRY(ctx, hipMemcpy(wf.data(), src, nn * sizeof(float), hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < nn; ++e) w[e] = wf[e];
  } else {
    HIP_TRY(ctx, hipMemcpy(w.data(), ctx->fac_wsd + D.fac_off + (int64_t)shift * nn, nn * sizeof(double),
                           hipMemcpyDeviceToHost));
  }
  for (int c = 0; c < np; ++c)
    for (int r = 0; r < np; ++r) lu[r + (int64_t)c * ldlu] = w[r + (int64_t)c * np];
  HIP_TRY(ctx, hipMemcpy(ipiv, ctx->fac_wsi + D.ipiv_ioff + (int64_t)shift * np, np * sizeof(int32_t),
                         hipMemcpyDeviceToHost));
  return PFM_OK;
}

int pfm_tune_import(pfm_ctx *ctx, const char *text) {
  if (!ctx || !text) return PFM_ERR_INVALID;
  std::map<uint64_t, int> t;
  const char *p = text;
  while (*p) {
    unsigned long long key;
    int pol, used = 0;
    if (sscanf(p, "%llu %d%n", &key, &pol, &used) != 2) break;
    if (pol < 0 || pol >= kNumPolicies) return set_err(ctx, PFM_ERR_INVALID, "tuning table: bad policy %d", pol);
    t[(uint64_t)key] = pol;
    p += used;
    while (*p == '\n' || *p == ' ' || *p == '\r') ++p;
  }
  if (*p) return set_err(ctx, PFM_ERR_INVALID, "tuning table: unreadable line");
  ctx->tuned = t;
  return PFM_OK;
}

}  // extern "C"
