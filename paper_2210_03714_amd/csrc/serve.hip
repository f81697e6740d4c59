// libpfm serving runtime: continuous batching of independent requests over
// pfm_eval_batched (pfm_srv_* in pfm.h).
//
// One scheduler thread owns `lanes` lanes; a lane is a context (its own
// workspace and pinned staging) plus a stream and a
// completion event, so up to `lanes` batches are in flight on the GPU at
// once.  Each scheduler pass:
//   1. retires lanes whose completion event has fired: their requests
//      become done (latency stamped), and their input copies are freed;
//   2. admits pending requests in arrival order while their resident bytes
//      (A, V, outputs) fit the resident share of the budget, allocating the
//      buffers from a device pool;
//   3. for every idle lane, takes the group of the oldest admitted request
//      (for an express lane: the oldest of real dimension <= 512)
//      (requests of one group share f, m, prec, dtype, mode and size bucket;
//      tolerances may differ), fills a batch in arrival order up to max_batch requests and
//      the lane's workspace share, copies the inputs into the resident
//      buffers on the lane's stream and calls pfm_eval_batched on the lane.
// Submitting only appends to the pending queue under the lock; the
// scheduler drops the lock while it launches, so submissions never wait on
// the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pfm.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Device memory pool: power-of-two size classes carved from 256 MiB chunks
// (larger requests get their own chunk); blocks return to their class's free
// list and chunks are kept until the server stops, so the scheduler never
// calls hipFree (which would wait for the whole device).
class DevicePool {
 public:
  explicit DevicePool(int device) : device_(device) {}
  ~DevicePool() {
    for (void *c : chunks_) (void)hipFree(c);
  }
  static size_t round(size_t b) {
    size_t s = 256;
    while (s < b) s <<= 1;
    return s;
  }
  void *alloc(size_t bytes) {
    const size_t s = round(bytes);
    auto &fl = free_[s];
    if (!fl.empty()) {
      void *p = fl.back();
      fl.pop_back();
      return p;
    }
    if (s >= kChunk) {
      void *p = nullptr;
      if (hipMalloc(&p, s) != hipSuccess) return nullptr;
      chunks_.push_back(p);
      return p;
    }
    if (cur_ == nullptr || cur_off_ + s > kChunk) {
      void *p = nullptr;
      if (hipMalloc(&p, kChunk) != hipSuccess) return nullptr;
      chunks_.push_back(p);
      cur_ = (char *)p;
      cur_off_ = 0;
    }
    void *p = cur_ + cur_off_;
    cur_off_ += s;
    return p;
  }
  void free(void *p, size_t bytes) {
    if (p) free_[round(bytes)].push_back(p);
  }

 private:
  static constexpr size_t kChunk = size_t(256) << 20;
  int device_;
  std::vector<void *> chunks_;
  std::map<size_t, std::vector<void *>> free_;
  char *cur_ = nullptr;
  size_t cur_off_ = 0;
};

enum ReqState { kPending = 0, kAdmitted = 1, kRunning = 2, kDone = 3, kFailed = 4 };

struct Req {
  uint64_t id = 0;
  pfm_problem prob{};  // caller's pointers (A, V)
  int f = 0, m = 0, prec = 0, dtype = 0;
  double tol = 0.0;
  int state = kPending;
  size_t esz = 8;                     // element size
  size_t a_bytes = 0, v_bytes = 0, o_bytes = 0;
  void *rA = nullptr, *rV = nullptr;  // resident copies (row-major, ld = n / p)
  void *rFe = nullptr, *rFp = nullptr;
  size_t ws = 0;                      // workspace estimate
  double t_submit = 0.0, t_done = 0.0;
  double t_admit = 0.0, t_dispatch = 0.0, t_launched = 0.0;  // admitted, handed to a lane, enqueued
  pfm_info info{};
  bool reported = false;
};

struct Lane {
  bool express = false;        // serves only requests of size bucket <= 1
  // a batch handed to the lane's launch thread, and its outcome
  std::vector<Req *> todo;
  bool has_todo = false, launched = false;
  int launch_rc = 0;
  std::thread th;
  std::condition_variable cv;
  pfm_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void *d_info = nullptr;
  pfm_info *h_info = nullptr;  // pinned
  int cap = 0;                 // info slots
  bool busy = false;
  std::vector<uint64_t> reqs;
};

// size bucket of the real dimension the kernels see (2n for complex): a
// batch runs as long as its largest member, so small requests are never
// batched with large ones
int size_bucket(const Req &r) {
  const int nk = r.dtype == PFM_C128 ? 2 * r.prob.n : r.prob.n;
  return nk <= 128 ? 0 : (nk <= 512 ? 1 : 2);
}

// requests that can share one call: tolerances may differ (each instance
// is planned with its own θ)
bool same_group(const Req &a, const Req &b) {
  return a.f == b.f && a.m == b.m && a.prec == b.prec && a.dtype == b.dtype &&
         (a.prob.p > 0) == (b.prob.p > 0) && size_bucket(a) == size_bucket(b);
}

}  // namespace

struct pfm_server {
  int device = 0;
  int max_batch = 64;
  size_t budget = 0, res_budget = 0, lane_budget = 0;
  size_t resident = 0, peak_resident = 0;
  uint64_t next_id = 1, n_submitted = 0, n_done = 0, n_batches = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> pending;     // arrival order, not yet admitted
  std::deque<uint64_t> admitted;    // admitted, not yet dispatched (arrival order)
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<Lane> lanes;  // lanes hold threads and condition variables: built in place
  DevicePool *pool = nullptr;
  std::thread th;
  bool stop = false;
  int fatal = 0;
  double launch_s = 0.0;  // host time spent launching batches (all lanes)
};

namespace {

// the lock is held by the caller
void retire(pfm_server *S, Lane &L, bool ok) {
  const double t = now_s();
  for (size_t i = 0; i < L.reqs.size(); ++i) {
    auto it = S->reqs.find(L.reqs[i]);
    if (it == S->reqs.end()) continue;
    Req &r = it->second;
    r.state = ok ? kDone : kFailed;
    r.t_done = t;
    if (ok) r.info = L.h_info[i];
    S->pool->free(r.rA, r.a_bytes);
    S->pool->free(r.rV, r.v_bytes);
    r.rA = r.rV = nullptr;
    S->resident -= r.a_bytes + r.v_bytes;
    ++S->n_done;
  }
  L.reqs.clear();
  L.busy = false;
}

bool admit_one(pfm_server *S, Req &r) {
  const size_t need = r.a_bytes + r.v_bytes + r.o_bytes * ((r.f & PFM_EXP ? 1 : 0) + (r.f & PFM_PHI1 ? 1 : 0));
  if (S->resident + need > S->res_budget) return false;
  r.rA = S->pool->alloc(r.a_bytes);
  if (r.v_bytes) r.rV = S->pool->alloc(r.v_bytes);
  if (r.f & PFM_EXP) r.rFe = S->pool->alloc(r.o_bytes);
  if (r.f & PFM_PHI1) r.rFp = S->pool->alloc(r.o_bytes);
  if (!r.rA || (r.v_bytes && !r.rV) || ((r.f & PFM_EXP) && !r.rFe) || ((r.f & PFM_PHI1) && !r.rFp)) {
    S->pool->free(r.rA, r.a_bytes);
    S->pool->free(r.rV, r.v_bytes);
    S->pool->free(r.rFe, r.o_bytes);
    S->pool->free(r.rFp, r.o_bytes);
    r.rA = r.rV = r.rFe = r.rFp = nullptr;
    return false;
  }
  S->resident += need;
  S->peak_resident = std::max(S->peak_resident, S->resident);
  r.state = kAdmitted;
  r.t_admit = now_s();
  return true;
}

// Launch one batch on lane L (lock not held; the batch's requests are
// already marked running, so no one else touches them).
int launch(pfm_server *S, Lane &L, std::vector<Req *> &batch) {
  const int nb = (int)batch.size();
  std::vector<pfm_problem> probs(nb);
  std::vector<double> tols(nb);
  for (int i = 0; i < nb; ++i) {
    Req &r = *batch[i];
    const int n = r.prob.n, p = r.prob.p;
    // inputs into the resident buffers (rows packed: ld = n, or p for V)
    if (hipMemcpy2DAsync(r.rA, (size_t)n * r.esz, r.prob.A, (size_t)r.prob.lda * r.esz, (size_t)n * r.esz, n,
                         hipMemcpyDeviceToDevice, L.stream) != hipSuccess)
      return PFM_ERR_HIP;
    if (p > 0 && hipMemcpy2DAsync(r.rV, (size_t)p * r.esz, r.prob.V, (size_t)r.prob.ldv * r.esz,
                                  (size_t)p * r.esz, n, hipMemcpyDeviceToDevice, L.stream) != hipSuccess)
      return PFM_ERR_HIP;
    tols[i] = r.tol;
    pfm_problem &q = probs[i];
    q.n = n;
    q.p = p;
    q.lda = n;
    q.ldv = p;
    q.ldf = p > 0 ? p : n;
    q.A = r.rA;
    q.V = r.rV;
    q.F_exp = r.rFe;
    q.F_phi1 = r.rFp;
  }
  if (nb > L.cap) {
    if (L.d_info) (void)hipFree(L.d_info);
    if (L.h_info) (void)hipHostFree(L.h_info);
    L.d_info = nullptr;
    L.h_info = nullptr;
    L.cap = 0;
    if (hipMalloc(&L.d_info, sizeof(pfm_info) * S->max_batch) != hipSuccess) return PFM_ERR_HIP;
    if (hipHostMalloc((void **)&L.h_info, sizeof(pfm_info) * S->max_batch, hipHostMallocDefault) != hipSuccess)
      return PFM_ERR_HIP;
    L.cap = S->max_batch;
  }
  const Req &r0 = *batch[0];
  int rc = pfm_eval_batched_tols(L.ctx, r0.f, r0.m, tols.data(), r0.tol, r0.prec, r0.dtype, nb, probs.data(),
                                 (pfm_info *)L.d_info, -1, L.stream);
  if (rc) return rc;
  if (hipMemcpyAsync(L.h_info, L.d_info, sizeof(pfm_info) * nb, hipMemcpyDeviceToHost, L.stream) != hipSuccess)
    return PFM_ERR_HIP;
  if (hipEventRecord(L.done, L.stream) != hipSuccess) return PFM_ERR_HIP;
  return PFM_OK;
}

// One thread per lane: launches the batches the scheduler hands over, so
// that one lane whose call waits (to grow its workspace, or for the step
// count of a large action) never holds up the dispatch of the others.
void lane_main(pfm_server *S, Lane *L) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    L->cv.wait(lk, [&] { return L->has_todo || (S->stop && !L->busy); });
    if (!L->has_todo) break;
    std::vector<Req *> batch;
    batch.swap(L->todo);
    lk.unlock();
    const double t0 = now_s();
    const int rc = launch(S, *L, batch);
    const double t1 = now_s();
    lk.lock();
    S->launch_s += t1 - t0;
    for (Req *r : batch) r->t_launched = t1;
    L->has_todo = false;
    L->launch_rc = rc;
    L->launched = true;
    S->cv.notify_all();
  }
}

void scheduler(pfm_server *S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progress = false;
    // 1. completions
    for (Lane &L : S->lanes) {
      if (!L.busy || !L.launched) continue;
      if (L.launch_rc) {
        retire(S, L, false);
        S->fatal = L.launch_rc;
        progress = true;
        continue;
      }
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipSuccess) {
        retire(S, L, true);
        progress = true;
      } else if (q != hipErrorNotReady) {
        retire(S, L, false);
        S->fatal = PFM_ERR_HIP;
        progress = true;
      }
    }
    // 2. admission in arrival order
    while (!S->pending.empty()) {
      Req &r = S->reqs[S->pending.front()];
      if (!admit_one(S, r)) break;
      S->admitted.push_back(r.id);
      S->pending.pop_front();
      progress = true;
    }
    // 3. dispatch to idle lanes: the group of the oldest admitted request
    //    (express lanes: of the oldest admitted request of size bucket <= 1)
    for (Lane &L : S->lanes) {
      if (L.busy || S->admitted.empty()) continue;
      const Req *hp = nullptr;
      for (uint64_t id : S->admitted) {
        const Req &r = S->reqs[id];
        if (!L.express || size_bucket(r) <= 1) {
          hp = &r;
          break;
        }
      }
      if (!hp) continue;
      std::vector<Req *> batch;
      const Req &head = *hp;
      const double td = now_s();
      size_t ws = 0;
      std::deque<uint64_t> rest;
      for (uint64_t id : S->admitted) {
        Req &r = S->reqs[id];
        if ((int)batch.size() < S->max_batch && same_group(r, head) && (batch.empty() || ws + r.ws <= S->lane_budget)) {
          batch.push_back(&r);
          ws += r.ws;
          r.state = kRunning;
          r.t_dispatch = td;
          L.reqs.push_back(id);
        } else {
          rest.push_back(id);
        }
      }
      S->admitted.swap(rest);
      L.busy = true;
      L.launched = false;
      L.todo.swap(batch);
      L.has_todo = true;
      ++S->n_batches;
      L.cv.notify_one();
      progress = true;
    }
    bool busy = false;
    for (Lane &L : S->lanes) busy |= L.busy;
    if (S->stop && S->pending.empty() && S->admitted.empty() && !busy) {
      for (Lane &L : S->lanes) L.cv.notify_one();
      break;
    }
    if (!progress) {
      // idle: wake on a submission, or poll the lanes again shortly
      S->cv.wait_for(lk, std::chrono::microseconds(busy ? 20 : 2000));
    }
  }
}

size_t elem_size(int dtype) { return dtype == PFM_C128 ? 16 : 8; }

}  // namespace

extern "C" {

int pfm_srv_start(pfm_server **out, int device, int lanes, size_t budget, int max_batch) {
  if (!out || lanes < 1 || lanes > 16 || budget == 0 || max_batch < 1) return PFM_ERR_INVALID;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return PFM_ERR_HIP;
  pfm_server *S = new pfm_server();
  S->device = device;
  S->max_batch = max_batch;
  S->budget = budget;
  S->res_budget = budget / 2;
  S->lane_budget = budget / 2 / lanes;
  S->pool = new DevicePool(device);
  for (int l = 0; l < lanes; ++l) S->lanes.emplace_back();
  // with two or more lanes, a third of them (at least one) are express
  // lanes for requests of real dimension <= 512, so that those never wait
  // behind batches of large ones
  const int nexp = lanes >= 2 ? std::max(1, lanes / 3) : 0;
  for (int l = 0; l < nexp; ++l) S->lanes[l].express = true;
  for (Lane &L : S->lanes) {
    if (pfm_create(&L.ctx, device, S->lane_budget) != PFM_OK || pfm_set_graphs(L.ctx, 0) != PFM_OK ||
        hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
      pfm_srv_stop(S);
      return PFM_ERR_HIP;
    }
  }
  for (Lane &L : S->lanes) L.th = std::thread(lane_main, S, &L);
  S->th = std::thread(scheduler, S);
  *out = S;
  return PFM_OK;
}

int pfm_srv_stop(pfm_server *S) {
  if (!S) return PFM_ERR_INVALID;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  {
    std::lock_guard<std::mutex> g(S->mu);
    for (Lane &L : S->lanes) L.cv.notify_all();
  }
  for (Lane &L : S->lanes)
    if (L.th.joinable()) L.th.join();
  (void)hipSetDevice(S->device);
  for (Lane &L : S->lanes) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    if (L.ctx) pfm_destroy(L.ctx);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    if (L.d_info) (void)hipFree(L.d_info);
    if (L.h_info) (void)hipHostFree(L.h_info);
  }
  delete S->pool;
  delete S;
  return PFM_OK;
}

int pfm_srv_submit(pfm_server *S, const pfm_problem *pr, int f, int m, double tol, int prec, int dtype,
                   uint64_t *ticket) {
  if (!S || !pr || !ticket) return PFM_ERR_INVALID;
  if (pr->n < 1 || pr->p < 0 || !pr->A || pr->lda < pr->n || (pr->p > 0 && (!pr->V || pr->ldv < pr->p)))
    return PFM_ERR_INVALID;
  if (f & PFM_PHI2) return PFM_ERR_UNSUPPORTED;  // served: exp and phi1
  if (f < 1 || f > 3 || !(tol > 0.0 && tol < 1.0)) return PFM_ERR_INVALID;
  if (prec != PFM_FP64 && prec != PFM_MIXED) return PFM_ERR_INVALID;
  if (dtype != PFM_R64 && dtype != PFM_C128) return PFM_ERR_INVALID;
  Req r;
  r.prob = *pr;
  r.f = f;
  r.m = m;
  r.tol = tol;
  r.prec = prec;
  r.dtype = dtype;
  r.esz = elem_size(dtype);
  const size_t n = pr->n, p = pr->p;
  r.a_bytes = n * n * r.esz;
  r.v_bytes = p * n * r.esz;
  r.o_bytes = (p > 0 ? n * p : n * n) * r.esz;
  pfm_problem q = *pr;
  r.ws = pfm_workspace_bytes(f, m, prec, dtype, 1, &q);
  if (r.ws == 0) return PFM_ERR_UNSUPPORTED;
  const size_t need = r.a_bytes + r.v_bytes + 2 * r.o_bytes;
  if (r.ws > S->lane_budget || need > S->res_budget) return PFM_ERR_BUDGET;
  r.t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) return PFM_ERR_INVALID;
    r.id = S->next_id++;
    *ticket = r.id;
    S->pending.push_back(r.id);
    S->reqs.emplace(r.id, r);
    ++S->n_submitted;
  }
  S->cv.notify_one();
  return PFM_OK;
}

int pfm_srv_poll(pfm_server *S, uint64_t ticket, pfm_info *info, double *latency) {
  if (!S) return PFM_ERR_INVALID;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return PFM_ERR_INVALID;
  const Req &r = it->second;
  if (r.state == kFailed) return PFM_ERR_HIP;
  if (r.state != kDone) return 1;
  if (info) *info = r.info;
  if (latency) *latency = r.t_done - r.t_submit;
  return PFM_OK;
}

int pfm_srv_drain(pfm_server *S, int max, uint64_t *tickets, double *latency, int32_t *status) {
  if (!S || max < 0 || (max > 0 && !tickets)) return PFM_ERR_INVALID;
  std::lock_guard<std::mutex> g(S->mu);
  int k = 0;
  for (auto &kv : S->reqs) {
    if (k >= max) break;
    Req &r = kv.second;
    if ((r.state == kDone || r.state == kFailed) && !r.reported) {
      r.reported = true;
      tickets[k] = r.id;
      if (latency) latency[k] = r.t_done - r.t_submit;
      if (status) status[k] = r.state == kDone ? r.info.status : -1;
      ++k;
    }
  }
  return k;
}

int pfm_srv_timing(pfm_server *S, uint64_t ticket, double *parts) {
  if (!S || !parts) return PFM_ERR_INVALID;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return PFM_ERR_INVALID;
  const Req &r = it->second;
  if (r.state != kDone && r.state != kFailed) return 1;
  parts[0] = r.t_admit - r.t_submit;
  parts[1] = r.t_dispatch - r.t_admit;
  // a batch whose launch failed is retired without a launch stamp
  const double tl = r.t_launched > 0.0 ? r.t_launched : r.t_done;
  parts[2] = tl - r.t_dispatch;
  parts[3] = r.t_done - tl;
  return PFM_OK;
}

int pfm_srv_fetch(pfm_server *S, uint64_t ticket, int which, void *dst, int64_t ldd) {
  if (!S || !dst) return PFM_ERR_INVALID;
  Req r;
  {
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second.state != kDone) return PFM_ERR_INVALID;
    r = it->second;
  }
  const void *src = which == PFM_EXP ? r.rFe : (which == PFM_PHI1 ? r.rFp : nullptr);
  if (!src) return PFM_ERR_INVALID;
  const size_t cols = r.prob.p > 0 ? r.prob.p : r.prob.n;
  if (ldd < (int64_t)cols) return PFM_ERR_INVALID;
  (void)hipSetDevice(S->device);
  if (hipMemcpy2D(dst, (size_t)ldd * r.esz, src, cols * r.esz, cols * r.esz, r.prob.n, hipMemcpyDeviceToDevice) !=
      hipSuccess)
    return PFM_ERR_HIP;
  return PFM_OK;
}

int pfm_srv_release(pfm_server *S, uint64_t ticket) {
  if (!S) return PFM_ERR_INVALID;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end() || (it->second.state != kDone && it->second.state != kFailed)) return PFM_ERR_INVALID;
  Req &r = it->second;
  const int nf = (r.f & PFM_EXP ? 1 : 0) + (r.f & PFM_PHI1 ? 1 : 0);
  S->pool->free(r.rFe, r.o_bytes);
  S->pool->free(r.rFp, r.o_bytes);
  S->resident -= r.o_bytes * nf;
  S->reqs.erase(it);
  S->cv.notify_one();
  return PFM_OK;
}

int pfm_srv_stats(pfm_server *S, uint64_t *submitted, uint64_t *done, uint64_t *batches, uint64_t *resident,
                  uint64_t *peak, double *launch_s) {
  if (!S) return PFM_ERR_INVALID;
  std::lock_guard<std::mutex> g(S->mu);
  if (launch_s) *launch_s = S->launch_s;
  if (submitted) *submitted = S->n_submitted;
  if (done) *done = S->n_done;
  if (batches) *batches = S->n_batches;
  if (resident) *resident = S->resident;
  if (peak) *peak = S->peak_resident;
  return S->fatal;
}

}  // extern "C"
