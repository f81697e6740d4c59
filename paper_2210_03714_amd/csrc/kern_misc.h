// Norm/plan, output store, info and self-test kernels.
#pragma once
#include "kern_common.h"
#include "pfm.h"

namespace pfm {

// eta = ||A||_1 (max column sum of |a_ij|; |z| for complex), then the plan of
// §1: s = smallest s >= 0 with eta 2^-s <= θ (full matrix) or
// N = max(1, ceil(eta / θ)) (action).  Three launches:
//   plan_init_kernel   (batch / 256 blocks): clear the plan records;
//   norm_kernel        (64-column chunk x instance): each column's sum in
//                      four row partitions (rows congruent mod 4, in order),
//                      combined in a fixed order, then the chunk's max folded
//                      into eta with an integer atomicMax on the bit pattern
//                      (eta >= 0, and NaN patterns order above +inf), so the
//                      result does not depend on scheduling;
//   plan_finish_kernel (batch / 256 blocks): s or N from eta.
__global__ void __launch_bounds__(256)
plan_init_kernel(PlanRec *__restrict__ plan, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  PlanRec P;
  P.s = 0;
  P.status = 0;
  P.bad_shift = 0x7fffffff;
  P.ir_iters = 0;
  P.route = 0;
  P.pad_ = 0;
  P.eta = 0.0;
  P.resid = 0.0;
  plan[i] = P;
}

__global__ void __launch_bounds__(256)
norm_kernel(const InstDesc *__restrict__ inst, PlanRec *__restrict__ plan) {
  __shared__ double part[4][64];
  const int ii = blockIdx.y;
  const InstDesc D = inst[ii];
  const int n = D.emb ? D.hn : D.n;  // the caller's matrix
  const int c0 = blockIdx.x * 64;
  if (c0 >= n) return;
  const int t = threadIdx.x, cl = t & 63, g = t >> 6;
  const int c = c0 + cl;
  double s = 0.0;
  if (c < n) {
    if (D.cin) {
      for (int r = g; r < n; r += 4) {
        const double *z = D.Ain + 2 * ((int64_t)r * D.ldin + c);
        s += hypot(z[0], z[1]);
      }
    } else {
      for (int r = g; r < n; r += 4) s += fabs(D.Ain[(int64_t)r * D.ldin + c]);
    }
  }
  part[g][cl] = s;
  __syncthreads();
  if (t < 64) {
    double v = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
    if (isnan(v)) v = __builtin_nan("");  // one canonical NaN
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v, off);
      v = (isnan(o) || o > v) ? o : v;
    }
    if (t == 0)
      atomicMax(reinterpret_cast<unsigned long long *>(&plan[ii].eta), (unsigned long long)__double_as_longlong(v));
  }
}

__global__ void __launch_bounds__(256)
plan_finish_kernel(const InstDesc *__restrict__ inst, PlanRec *__restrict__ plan, int batch, int action,
                   int force_plan, int unscaled) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const double theta = inst[i].theta;
  PlanRec P = plan[i];
  const double eta = P.eta;
  const bool bad = !isfinite(eta);
  if (bad) {
    P.eta = __builtin_nan("");
    P.status = 2;
  }
  int plan_v;
  if (force_plan >= 0) {
    plan_v = action ? (force_plan < 1 ? 1 : force_plan) : force_plan;
  } else if (bad) {
    plan_v = action ? 1 : 0;
  } else if (action) {
    const double q = ceil(eta / theta);
    plan_v = q < 1.0 ? 1 : (q > 1e9 ? 1000000000 : (int)q);
  } else {
    int s = 0;
    while (ldexp(eta, -s) > theta && s < 1023) ++s;
    plan_v = s;
  }
  if (unscaled) {  // a function without a scaling identity: s = 0
    plan_v = 0;
    if (!bad && eta > theta) P.status |= 16;  // PFM_OUT_OF_RANGE
  }
  P.s = plan_v;
  plan[i] = P;
}

// Copy the final R / Phi (column-major, npad) to the caller's row-major
// outputs, through a 32 x 32 LDS transpose.  Embedded instances: the first
// block column holds [Re R; Im R]; complex outputs are interleaved, a real
// output (conjugate pair on real A) takes the top half.  Grid: x = tile,
// y = instance.
__global__ void __launch_bounds__(256)
store_full_kernel(const InstDesc *__restrict__ inst, const PlanRec *__restrict__ plan,
                  const double *__restrict__ wsd, int want_exp, int want_phi, int want_phi2) {
  __shared__ double tile[2][32][33];
  const int ii = blockIdx.y;
  const InstDesc D = inst[ii];
  const int np = D.npad;
  const int n = D.emb ? D.hn : D.n;
  const int tn = (n + 31) / 32;
  const int tix = blockIdx.x;
  if (tix >= tn * tn) return;
  const int r0 = (tix % tn) * 32, c0 = (tix / tn) * 32;
  const int s = plan[ii].s;
  if (plan[ii].status & PFM_NOT_COMPUTED) return;
  const int64_t nn = (int64_t)np * np;
  const int t = threadIdx.x;
  const bool cplx_out = D.emb && D.cin;
  for (int which = 0; which < 3; ++which) {
    if (which == 0 && !want_exp) continue;
    if (which == 1 && !want_phi) continue;
    if (which == 2 && !want_phi2) continue;
    const double *src = wsd + D.r_off + (which * 2 + (s & 1)) * nn;
    double *dst = which == 2 ? D.Fq : (which ? D.Fp : D.Fe);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + (t & 7) * 4 + u, c = c0 + (t >> 3);
      const bool ok = r < n && c < n;
      tile[0][(t & 7) * 4 + u][t >> 3] = ok ? src[r + (int64_t)c * np] : 0.0;
      if (cplx_out) tile[1][(t & 7) * 4 + u][t >> 3] = ok ? src[r + D.hn + (int64_t)c * np] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + (t >> 3), c = c0 + (t & 7) * 4 + u;
      if (r < n && c < n) {
        if (cplx_out) {
          dst[2 * ((int64_t)r * D.ldf + c)] = tile[0][t >> 3][(t & 7) * 4 + u];
          dst[2 * ((int64_t)r * D.ldf + c) + 1] = tile[1][t >> 3][(t & 7) * 4 + u];
        } else {
          dst[(int64_t)r * D.ldf + c] = tile[0][t >> 3][(t & 7) * 4 + u];
        }
      }
    }
    __syncthreads();
  }
}

// E = emb(A) = [[Re A, -Im A], [Im A, Re A]] row-major (2 hn)^2 for embedded
// instances (a real A has Im A = 0).  Grid: x = 32x32 tile of E, y = instance.
__global__ void __launch_bounds__(256)
embed_kernel(const InstDesc *__restrict__ inst, double *__restrict__ wsd) {
  const int ii = blockIdx.y;
  const InstDesc D = inst[ii];
  if (!D.emb) return;
  const int n = D.n, hn = D.hn;
  const int tn = (n + 31) / 32;
  const int tix = blockIdx.x;
  if (tix >= tn * tn) return;
  const int r0 = (tix / tn) * 32, c0 = (tix % tn) * 32;
  double *E = wsd + D.e_off;
  const int t = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = r0 + (t >> 3), c = c0 + (t & 7) * 4 + u;
    if (r < n && c < n) {
      const int rb = r >= hn, cb = c >= hn;
      const int ri = r - rb * hn, ci = c - cb * hn;
      double x, y;
      if (D.cin) {
        x = D.Ain[2 * ((int64_t)ri * D.ldin + ci)];
        y = D.Ain[2 * ((int64_t)ri * D.ldin + ci) + 1];
      } else {
        x = D.Ain[(int64_t)ri * D.ldin + ci];
        y = 0.0;
      }
      E[(int64_t)r * n + c] = (rb == cb) ? x : (rb ? y : -y);
    }
  }
}

// The route of every instance, from its plan, on the device (the host reads
// nothing back).  With |c_k| ||B||_1 <= 1/2 for every shift, each
// I - c_k B is strictly column diagonally dominant, partial pivoting would
// never interchange rows, and the inverses are formed by Gauss-Jordan:
//   - the multi-workgroup route (2) for instances that may take it (action or
//     complex above the threshold, or n > 512), with the dominance test on
//     the real matrix the kernels see (||emb(B)||_1 <= sqrt(2) ||B||_1);
//     an instance above 512 that fails it is not computed (no other route);
//   - the single-workgroup Gauss-Jordan route (1) where the call allows it;
//   - else the pivoting LU route (0).  The hybrid set of §4.3 has no LU-route
//     form: such an instance is not computed.
// Plans above the caps (kSCap squarings, kNCap steps) are not computed
// either.
__global__ void __launch_bounds__(256)
route_kernel(const InstDesc *__restrict__ inst, PlanRec *__restrict__ plan, int batch, int action, double cmax,
             int hybrid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const InstDesc D = inst[i];
  PlanRec P = plan[i];
  const bool finite = !(P.status & PFM_NONFINITE);
  const double bn = action ? P.eta / (double)(P.s > 1 ? P.s : 1) : ldexp(P.eta, -(P.s < 1023 ? P.s : 1023));
  const bool ln_dom = finite && cmax * bn * (D.emb ? 1.4142135623730951 : 1.0) <= 0.5;
  const bool dom = finite && cmax * bn <= 0.5;
  int route = 0;
  if (D.rflags & kRfLarge) {
    route = 2;
    if (!ln_dom) P.status |= PFM_NOT_COMPUTED;
  } else if ((D.rflags & kRfMayLn) && ln_dom) {
    route = 2;
  } else if ((D.rflags & kRfGj) && dom) {
    route = 1;
  }
  if (hybrid && route == 0 && !action) P.status |= PFM_NOT_COMPUTED;  // the action's LU route adds the polynomial
  if (action ? P.s > kNCap : P.s > kSCap) P.status |= PFM_NOT_COMPUTED;
  P.route = route;
  plan[i] = P;
}

struct InfoRec {  // mirrors pfm_info
  int32_t status, plan, order, ir_iters, bad_shift, route;
  double norm1, theta, resid;
};

__global__ void info_kernel(const InstDesc *__restrict__ inst, const PlanRec *__restrict__ plan,
                            InfoRec *__restrict__ info, int batch, int order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const PlanRec P = plan[i];
  InfoRec r;
  r.status = P.status;
  r.plan = P.s;
  r.order = order;
  r.ir_iters = P.ir_iters;
  r.bad_shift = P.bad_shift == 0x7fffffff ? -1 : P.bad_shift;
  r.route = P.route;
  r.norm1 = P.eta;
  r.theta = inst[i].theta;
  r.resid = P.resid;
  info[i] = r;
}

// One 16x16x4 FP64 MFMA on known operands: A[i][k] = 4 i + k + 1,
// B[k][j] = 100 (k + 1) + j; lane l writes its four accumulator values.
__global__ void selftest_mfma_kernel(double *out) {
  const int l = threadIdx.x, i16 = l & 15, g = l >> 4;
  const double a = 4.0 * i16 + g + 1.0;
  const double b = 100.0 * (g + 1) + i16;
  v4d acc = mfma16(a, b, zero4());
#pragma unroll
  for (int v = 0; v < 4; ++v) out[l * 4 + v] = acc[v];
}

// The same check for v_mfma_f32_16x16x4_f32.
__global__ void selftest_mfma32_kernel(double *out) {
  const int l = threadIdx.x, i16 = l & 15, g = l >> 4;
  const float a = 4.0f * i16 + g + 1.0f;
  const float b = 100.0f * (g + 1) + i16;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  acc = mfma16(a, b, acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) out[l * 4 + v] = acc[v];
}

}  // namespace pfm
