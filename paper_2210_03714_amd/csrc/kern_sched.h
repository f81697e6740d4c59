// Squaring levels beyond the ones launched one by one: a persistent launch
// over a device-built queue of (level, instance, tile) tasks.
//
// The host does not read the plans back, so it cannot know how many
// squarings (§1) the instances need.  It launches the first L levels one
// launch per level (every listed instance's tiles; a tile of an instance with
// s < level returns at once) and then this queue for levels L + 1 .. s of
// every instance, whatever s is:
//
//   sq_queue_kernel    one workgroup: sorts the group's instances by s
//                      (descending; counting sort, ties in any order), the
//                      prefix sums of their tile counts in that order, and
//                      the first task of every level, then resets the queue
//                      head and the per-instance tile counters.  Level j's
//                      tasks are the tiles of the instances with s >= j,
//                      which in that order are a prefix of the list.
//   sq_persist_kernel  a grid of at most the resident workgroups: each
//                      takes the next task index with an atomic add, maps it
//                      to (level, instance, tile) by two binary searches,
//                      waits until every tile of that instance's previous
//                      level is done (its counter), computes the tile and
//                      counts it done.  It leaves when the index passes the
//                      last task.
//
// The tasks are ordered level by level, so a task only ever waits for tasks
// with smaller indices, which were taken earlier by workgroups that were
// running then and themselves wait only for smaller indices: the unfinished
// task with the smallest index always has its inputs, and the queue drains
// however many workgroups are resident at once (no workgroup waits for a
// workgroup that has not started).  Every wait is bounded; one that gives up
// sets a flag that pfm_check reports (PFM_ERR_DEVICE), every later wait of
// the launch then gives up at once, and the tiles are computed anyway, so the
// kernel always ends.
//
// Memory ordering across workgroups (and XCDs): the producer's threads fence
// at agent scope after their stores and before the barrier after which one
// thread adds to the counter; the consumer reads the counter with an
// agent-scope acquire load and every thread fences (acquire, agent) after the
// barrier that follows, before loading the operands.
#pragma once
#include "kern_square.h"

namespace pfm {

struct SqQueue {
  unsigned long long head;  // next task index
  long long total;          // tasks in the queue
  int32_t smax;             // largest level
  int32_t first;            // first level in the queue
  int32_t ng;               // instances in the group
  int32_t pad_;
};

// Output tiles of one level of instance D (R and, with phi1, Phi).
__host__ __device__ inline int sq_tiles(int npad, int ncol, int tile, int nw) {
  return ((npad + tile - 1) / tile) * ((ncol + tile - 1) / tile) * nw;
}

constexpr int kQueueThreads = 256;

// Build the queue of levels first..s_i for the instances gl[0..ng) (tile
// edge `tile`, nw = 1 + want_phi products per level).  Arrays: ord[ng],
// pre[ng + 1], lstart[kSCap + 2], done[ng].
__global__ void __launch_bounds__(kQueueThreads)
sq_queue_kernel(const InstDesc *__restrict__ inst, const PlanRec *__restrict__ plan, const int *__restrict__ gl,
                int ng, int tile, int nw, int first, SqQueue *__restrict__ q, int *__restrict__ ord,
                long long *__restrict__ pre, long long *__restrict__ lstart, int *__restrict__ done) {
  __shared__ int hist[kSCap + 2];
  __shared__ int pos[kSCap + 2];
  __shared__ long long part[kQueueThreads];
  __shared__ int smax_s;
  const int t = threadIdx.x;
  for (int v = t; v < kSCap + 2; v += kQueueThreads) hist[v] = 0;
  if (t == 0) smax_s = 0;
  for (int r = t; r < ng; r += kQueueThreads) done[r] = 0;
  __syncthreads();
  // levels of instance r: s (0 if not computed), capped
  auto lev = [&](int r) -> int {
    const PlanRec &P = plan[gl[r]];
    if (P.status & PFM_NOT_COMPUTED) return 0;
    return P.s < 0 ? 0 : (P.s > kSCap ? kSCap : P.s);
  };
  for (int r = t; r < ng; r += kQueueThreads) {
    const int s = lev(r);
    atomicAdd(&hist[s], 1);
    atomicMax(&smax_s, s);
  }
  __syncthreads();
  if (t == 0) {  // start of each s in descending order
    int run = 0;
    for (int v = kSCap; v >= 0; --v) {
      pos[v] = run;
      run += hist[v];
    }
  }
  __syncthreads();
  for (int r = t; r < ng; r += kQueueThreads) ord[atomicAdd(&pos[lev(r)], 1)] = r;
  __syncthreads();
  // prefix sums of the tile counts in sorted order: each thread a chunk
  const int per = (ng + kQueueThreads - 1) / kQueueThreads;
  const int lo = t * per, hi = lo + per < ng ? lo + per : ng;
  long long sum = 0;
  for (int k = lo; k < hi; ++k) {
    const InstDesc &D = inst[gl[ord[k]]];
    sum += sq_tiles(D.npad, D.ncol, tile, nw);
  }
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    long long run = 0;
    for (int u = 0; u < kQueueThreads; ++u) {
      const long long v = part[u];
      part[u] = run;
      run += v;
    }
  }
  __syncthreads();
  long long run = part[t];
  for (int k = lo; k < hi; ++k) {
    pre[k] = run;
    const InstDesc &D = inst[gl[ord[k]]];
    run += sq_tiles(D.npad, D.ncol, tile, nw);
  }
  if (t == kQueueThreads - 1) pre[ng] = run;  // the last chunk ends at ng (or is empty and run = total)
  __syncthreads();
  if (t == 0) {
    const int smax = smax_s;
    // instances with s >= j: all but those with s < j
    int cnt = ng;
    for (int v = 0; v < first && v <= kSCap; ++v) cnt -= hist[v];
    long long acc = 0;
    lstart[first] = 0;
    for (int j = first; j <= smax; ++j) {
      acc += pre[cnt];
      lstart[j + 1] = acc;
      cnt -= hist[j];
    }
    q->head = 0ull;
    q->total = smax >= first ? acc : 0;
    q->smax = smax;
    q->first = first;
    q->ng = ng;
    q->pad_ = 0;
  }
}

constexpr long long kWaitSpins = 1ll << 22;  // bounded wait (seconds); after one gives up, the rest do at once

template <int TILE>
__global__ void __launch_bounds__(256, 2)
sq_persist_kernel(const InstDesc *__restrict__ inst, const PlanRec *__restrict__ plan, const int *__restrict__ gl,
                  int nw, SqQueue *__restrict__ q, const int *__restrict__ ord, const long long *__restrict__ pre,
                  const long long *__restrict__ lstart, int *__restrict__ done, double *__restrict__ wsd,
                  int *__restrict__ err) {
  __shared__ long long tsh;
  const int t = threadIdx.x;
  // written by sq_queue_kernel, earlier in stream order
  const long long total = q->total;
  const int first = q->first, smax = q->smax, ng = q->ng;
  // Thread 0 takes the next task index at the end of each iteration (and
  // once before the loop), in the same block as its completion count, so
  // that the loop has one thread-0 branch and one exit.  With a thread-0
  // branch at both ends of the body, the compiler threads one into the other
  // across the back edge and turns the body into an inner loop that the
  // other lanes of wave 0 repeat without thread 0 -- on the old index,
  // forever.  The index is read through readfirstlane, so the exit is a
  // scalar branch.
  if (t == 0) tsh = (long long)atomicAdd(&q->head, 1ull);
  __syncthreads();
  for (;;) {
    const long long tv = tsh;
    const long long tk =
        (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(tv >> 32)) << 32) |
                    (unsigned)__builtin_amdgcn_readfirstlane((int)(tv & 0xffffffffll)));
    if (tk >= total) break;
    // level: the last j with lstart[j] <= tk
    int lo = first, hi = smax;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (lstart[mid] <= tk) lo = mid;
      else hi = mid - 1;
    }
    const int j = lo;
    const long long loc = tk - lstart[j];
    // rank in sorted order: the last r with pre[r] <= loc
    int rl = 0, rh = ng - 1;
    while (rl < rh) {
      const int mid = (rl + rh + 1) >> 1;
      if (pre[mid] <= loc) rl = mid;
      else rh = mid - 1;
    }
    const int gs = ord[rl];
    const int ii = gl[gs];
    const InstDesc &D = inst[ii];
    const int per = sq_tiles(D.npad, D.ncol, TILE, 1);
    const int u = (int)(loc - pre[rl]);
    const int which = u / per, lt = u - which * per;
    const int need = (j - first) * per * nw;  // every tile of the instance's earlier queued levels
    if (need > 0) {
      if (t == 0) {
        long long spins = 0;
        while (__hip_atomic_load(&done[gs], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(2);
          ++spins;
          if (spins > kWaitSpins ||
              ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            atomicOr(err, 1);
            break;
          }
        }
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    sq_tile<0, TILE>(inst, SqTask{ii, lt + (which << 20)}, j, wsd, plan, 0.0, 0.0, 0.0, 0.0);
    __threadfence();
    __syncthreads();  // every thread's stores of the tile, and its read of tsh, are done
    if (t == 0) {
      atomicAdd(&done[gs], 1);
      tsh = (long long)atomicAdd(&q->head, 1ull);
    }
    __syncthreads();
  }
}

// Zero-fill (device memory a captured graph may reuse: no memset nodes).
__global__ void zero_ints_kernel(int *__restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace pfm
