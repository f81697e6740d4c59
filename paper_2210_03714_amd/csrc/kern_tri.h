// Tridiagonal A (§2.1, §5): the action f(A)V by the N-step recurrence with
// the round-off form of §4.3, A given by its three diagonals.
//
// I - c_k B is tridiagonal, so each shifted system costs one forward and one
// backward sweep (the paper's 8d-flop count, §2.1); the LU of every shifted
// matrix is formed once and reused by all N steps and all columns (§5.1).
// With ||B||_1 <= θ every I - c_k B is strictly column diagonally dominant
// (|c_k| ||B||_1 < 0.2 on the registered sets), so elimination without
// interchanges is the partial-pivoting LU.
//
// Layout (one thread per column of V, a wave per 64 consecutive columns of
// one instance, so every factor read is the same address in all lanes):
//   B:        sub[r] = B[r][r-1] (sub[0] = 0), dia[r], sup[r] = B[r][r+1]
//             (sup[d-1] = 0)
//   factors:  per shift k, l[r] = M[r][r-1] / u[r-1] (l[0] = 0) and
//             ui[r] = 1 / u[r], M = I - c_k B = L U
//   vectors:  per function slot, two ping-pong buffers and u_1 (phi1), each
//             d x p row-major (lanes read consecutive addresses)
//   checkpoints: the forward sweep's value at the end of every kTriL-row
//             chunk, per shift, [chunk][k][column]
// A step reads the input vector twice and writes the output once: the first
// pass runs the forward sweeps of all shifts and keeps only the chunk-end
// values; the second pass walks the chunks from the last, recomputes each
// chunk's forward values from its checkpoint in registers, and runs the
// backward sweep, accumulating a0 x + sum_k w_k x_k on the way.
#pragma once
#include "kern_common.h"

namespace pfm {

constexpr int kTriL = 8;         // rows per checkpoint chunk
constexpr int kTriTerms = 8;     // most shifts in a real set

struct TriDesc {
  const double *dl, *dd, *du, *V;
  double *Fe, *Fp;
  int64_t ldv, ldf;
  int32_t d, p;
  double theta;
  int64_t b_off;  // sub, dia, sup: 3 d
  int64_t f_off;  // factors: [k][l, ui][d]
  int64_t v_off;  // vectors: [slot][3][d][p]
  int64_t c_off;  // checkpoints: [slot][chunk][k][p]
  int32_t wave0;   // first wave of this instance in the step launch
  int32_t nwaves;  // its waves: functions x ceil(p / 64)
};

struct TriTerms {
  int32_t nterms, nf;
  int32_t fn[2];  // function of each slot: 0 exp, 1 phi1
  double a0e, a0p;
  double c[kTriTerms], we[kTriTerms], wp[kTriTerms];
};

// ||A||_1 (largest column sum |du[j-1]| + |dd[j]| + |dl[j]|, summed in that
// order) and N = max(1, ceil(eta / θ)); one workgroup per instance.
__global__ void __launch_bounds__(256)
tri_plan_kernel(const TriDesc *__restrict__ desc, PlanRec *__restrict__ plan, int force_plan) {
  __shared__ double red[4];
  __shared__ int bad[4];
  const int ii = blockIdx.x, t = threadIdx.x;
  const TriDesc D = desc[ii];
  double mx = 0.0;
  int nan = 0;
  for (int j = t; j < D.d; j += 256) {
    double s = fabs(D.dd[j]);
    if (j > 0) s += fabs(D.du[j - 1]);
    if (j + 1 < D.d) s += fabs(D.dl[j]);
    if (isnan(s)) nan = 1;
    else mx = fmax(mx, s);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off));
    nan |= __shfl_xor(nan, off);
  }
  if ((t & 63) == 0) {
    red[t >> 6] = mx;
    bad[t >> 6] = nan;
  }
  __syncthreads();
  if (t != 0) return;
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  nan = bad[0] | bad[1] | bad[2] | bad[3];
  PlanRec P;
  P.s = 1;
  P.status = 0;
  P.bad_shift = 0x7fffffff;
  P.ir_iters = 0;
  P.route = 3;
  P.pad_ = 0;
  P.eta = nan ? __builtin_nan("") : mx;
  P.resid = 0.0;
  const bool nonfinite = !isfinite(P.eta);
  if (nonfinite) P.status = 2;
  if (force_plan >= 0) {
    P.s = force_plan < 1 ? 1 : force_plan;
  } else if (!nonfinite) {
    const double q = ceil(P.eta / D.theta);
    P.s = q < 1.0 ? 1 : (q > 1e9 ? 1000000000 : (int)q);
  }
  plan[ii] = P;
}

// B = A / N and the LU of I - c_k B for every (instance, shift): one thread
// each, a sequential sweep down the diagonal.  A zero or non-finite pivot
// sets PFM_SINGULAR_SHIFT with the smallest such shift.
__global__ void __launch_bounds__(64)
tri_factor_kernel(const TriDesc *__restrict__ desc, PlanRec *__restrict__ plan, int batch, TriTerms T,
                  double *__restrict__ wsd) {
  const int gid = blockIdx.x * 64 + threadIdx.x;
  const int ii = gid / T.nterms, k = gid - ii * T.nterms;
  if (ii >= batch) return;
  const TriDesc D = desc[ii];
  const int d = D.d;
  const double Nd = (double)plan[ii].s;
  const double c = T.c[k];
  double *sub = wsd + D.b_off, *dia = sub + d, *sup = dia + d;
  double *l = wsd + D.f_off + (int64_t)k * 2 * d, *ui = l + d;
  if (k == 0) {
    for (int r = 0; r < d; ++r) {
      sub[r] = r > 0 ? D.dl[r - 1] / Nd : 0.0;
      dia[r] = D.dd[r] / Nd;
      sup[r] = r + 1 < d ? D.du[r] / Nd : 0.0;
    }
  }
  bool bad = false;
  double u = 1.0 - c * (D.dd[0] / Nd);
  bad |= !(u != 0.0 && isfinite(u));
  l[0] = 0.0;
  ui[0] = 1.0 / u;
  for (int r = 1; r < d; ++r) {
    const double mlo = -c * (D.dl[r - 1] / Nd);  // M[r][r-1]
    const double mup = -c * (D.du[r - 1] / Nd);  // M[r-1][r]
    const double lr = mlo / u;
    u = (1.0 - c * (D.dd[r] / Nd)) - lr * mup;
    bad |= !(u != 0.0 && isfinite(u));
    l[r] = lr;
    ui[r] = 1.0 / u;
  }
  if (bad) {
    atomicOr(&plan[ii].status, 1);
    atomicMin(&plan[ii].bad_shift, k);
  }
}

// All N steps of one column (lane) of one function slot; one wave per
// workgroup, 64 consecutive columns of one instance.  The instance's B and
// factor rows are staged through LDS in blocks of kTriRB rows (a coalesced
// load by the whole wave into the buffer not being read, at each block
// boundary); the sweeps read them as broadcasts.  The column's own values
// are read two chunks ahead in the forward pass and one chunk ahead in the
// backward pass.  fac is the read-only view of B and the factors; vws holds
// the vectors and checkpoints (disjoint parts of the same workspace).  Lanes
// past p repeat column p - 1 and so store what that lane stores.
constexpr int kTriRB = 64;                // rows per staged block (one per lane)

// Vector loads and stores through global (not flat) instructions: flat
// accesses also count against the LDS counter, so every wait for an LDS read
// would wait for the in-flight prefetches as well.
__device__ __forceinline__ double gld(const double *a) {
  return *(const __attribute__((address_space(1))) double *)a;
}
__device__ __forceinline__ void gst(double *a, double v) {
  *(__attribute__((address_space(1))) double *)a = v;
}
constexpr int kTriF = 3 + 2 * kTriTerms;  // sub, dia, sup, l_k, u_k

// NT: the number of shifts (4, 5 or 8), so that the sweeps of all shifts
// unroll without branches and their chains interleave.  Rows past d (the
// tail of the last chunk) are swept too, on the clamped last row's factors,
// and never stored.
template <int NT>
__global__ void __launch_bounds__(64)
tri_steps_kernel(const TriDesc *__restrict__ desc, int batch, const PlanRec *__restrict__ plan, TriTerms T,
                 const double *__restrict__ fac, double *__restrict__ vws) {
  __shared__ double fb[2][kTriF][kTriRB];
  const int lane = threadIdx.x;
  const int gw = blockIdx.x;
  int lo = 0, hi = batch - 1;  // the instance whose waves contain gw
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].wave0 <= gw) lo = mid;
    else hi = mid - 1;
  }
  const int ii = __builtin_amdgcn_readfirstlane(lo);
  const TriDesc D = desc[ii];
  const int d = D.d, p = D.p;
  constexpr int nt = NT;
  const int cpw = (p + 63) / 64;
  const int wl = gw - D.wave0;
  const int slot = wl / cpw;
  const int c0 = (wl - slot * cpw) * 64 + lane;
  // lanes past p repeat column p - 1 exactly (same inputs, same arithmetic),
  // so their stores write the values that lane writes: no store needs a mask
  const int c = c0 < p ? c0 : p - 1;
  const int fn = slot == 0 ? T.fn[0] : T.fn[1];
  const int N = plan[ii].s;
  const int nch = (d + kTriL - 1) / kTriL;
  const int nb = (d + kTriRB - 1) / kTriRB;
  const double *sub = fac + D.b_off, *dia = sub + d, *sup = dia + d;
  const double *lf = fac + D.f_off;
  const int64_t dp = (int64_t)d * p;
  double *vb = vws + D.v_off + (int64_t)slot * 3 * dp;
  double *u1 = vb + 2 * dp;
  double *ck = vws + D.c_off + (int64_t)slot * nch * nt * p;

  double nf[kTriF];
  auto fetch = [&](int blk) {
    const int r = blk * kTriRB + lane < d ? blk * kTriRB + lane : d - 1;
    nf[0] = sub[r];
    nf[1] = dia[r];
    nf[2] = sup[r];
#pragma unroll
    for (int k = 0; k < kTriTerms; ++k) {
      const bool on = k < nt;
      const int64_t o = (int64_t)(on ? k : 0) * 2 * d + r;
      nf[3 + k] = on ? lf[o] : 0.0;
      nf[3 + kTriTerms + k] = on ? lf[o + d] : 0.0;
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int f = 0; f < kTriF; ++f) fb[buf][f][lane] = nf[f];
  };
  fetch(0);
  put(0);
  __syncthreads();

#pragma unroll 1
  for (int j = 0; j < N; ++j) {
    const double *src = j == 0 ? D.V + c : vb + (int64_t)((j - 1) & 1) * dp + c;
    const int64_t lds = j == 0 ? D.ldv : p;
    double *dst = j == N - 1 ? (fn ? D.Fp : D.Fe) + c : vb + (int64_t)(j & 1) * dp + c;
    const int64_t ldd = j == N - 1 ? D.ldf : p;
    const bool first_phi = fn == 1 && j == 0;
    const double a0 = first_phi ? T.a0p : T.a0e;
    // rows outside [0, d) read sub[0], which is 0: the address is chosen,
    // not the value, so no load sits behind a branch
    auto xload = [&](int r) {
      const double *a = (r >= 0 && r < d) ? src + (int64_t)r * lds : sub;
      return gld(a);
    };

    // pass 1 (block 0 is staged in buffer 0): forward sweeps
    // z_r = y_r - l_r z_{r-1} of every shift, y = B x; keep z at the end of
    // each chunk that has a successor.  x is read two chunks ahead.
    {
      double z[kTriTerms];
#pragma unroll
      for (int k = 0; k < kTriTerms; ++k) z[k] = 0.0;
      double xm = 0.0, xg[kTriL], xn[kTriL], xnn[kTriL];
#pragma unroll
      for (int jj = 0; jj < kTriL; ++jj) {
        xg[jj] = xload(jj);
        xn[jj] = xload(kTriL + jj);
      }
#pragma unroll 1
      for (int b = 0; b < nb; ++b) {
        const int buf = b & 1;
#pragma unroll 1
        for (int g = 0; g < kTriRB / kTriL; ++g) {
          const int rg = b * kTriRB + g * kTriL;
          if (rg >= d) break;
#pragma unroll
          for (int jj = 0; jj < kTriL; ++jj) xnn[jj] = xload(rg + 2 * kTriL + jj);
#pragma unroll
          for (int jj = 0; jj < kTriL; ++jj) {
            const int lr = g * kTriL + jj;
            const double x0 = xg[jj];
            const double xp = jj + 1 < kTriL ? xg[jj + 1] : xn[0];
            const double y = fma(fb[buf][2][lr], xp, fma(fb[buf][0][lr], xm, fb[buf][1][lr] * x0));
#pragma unroll
            for (int k = 0; k < NT; ++k) z[k] = fma(-fb[buf][3 + k][lr], z[k], y);
            xm = x0;
          }
          {  // the last chunk's slot is written and never read
            double *cq = ck + (int64_t)(rg / kTriL) * nt * p + c;
#pragma unroll
            for (int k = 0; k < NT; ++k) gst(cq + (int64_t)k * p, z[k]);
          }
#pragma unroll
          for (int jj = 0; jj < kTriL; ++jj) {
            xg[jj] = xn[jj];
            xn[jj] = xnn[jj];
          }
        }
        if (b + 1 < nb) {
          fetch(b + 1);
          put(buf ^ 1);
          __syncthreads();
        }
      }
    }

    // pass 2 (block nb - 1 is staged): chunks from the last.  Per chunk, the
    // forward values of every shift from the chunk's checkpoints, then the
    // backward sweeps x_r = (z_r - s_r x_{r+1}) / u_r with
    // s_r = M[r][r+1] = -c_k sup[r], all shifts row by row (independent
    // chains side by side), and out_r = a0 x_r + sum_k w_k x_{k,r}.  The next
    // chunk's rows and checkpoints are read during the backward sweeps.
    double xc[NT], zc[NT];
    double xs[kTriL + 2];  // rows r0 - 1 .. r0 + kTriL of the current chunk
    double us[kTriL];      // u_1 on the chunk's rows (phi1 after its first step)
    const bool add_u1 = fn == 1 && j > 0;
    auto chunk_loads = [&](int q) {
#pragma unroll
      for (int jj = 0; jj < kTriL + 2; ++jj) xs[jj] = xload(q * kTriL - 1 + jj);
#pragma unroll
      for (int jj = 0; jj < kTriL; ++jj) {
        const int r = q * kTriL + jj;
        const double *a = (add_u1 && r < d) ? u1 + (int64_t)r * p + c : sub;
        us[jj] = gld(a);
      }
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const double *a = q > 0 ? ck + ((int64_t)(q - 1) * NT + k) * p + c : sub;
        zc[k] = gld(a);
      }
    };
    double wk[NT], sk[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      xc[k] = 0.0;
      wk[k] = first_phi ? T.wp[k] : T.we[k];
      sk[k] = -T.c[k];
    }
    chunk_loads(nch - 1);
    const double rN = (double)N;
#pragma unroll 1
    for (int b = nb - 1; b >= 0; --b) {
      const int buf = b & 1;
#pragma unroll 1
      for (int g = kTriRB / kTriL - 1; g >= 0; --g) {
        const int r0 = b * kTriRB + g * kTriL;
        if (r0 >= d) continue;
        const int q = r0 / kTriL;
        const int len = d - r0 < kTriL ? d - r0 : kTriL;
        double zz[NT][kTriL], ax[kTriL];
#pragma unroll
        for (int jj = 0; jj < kTriL; ++jj) {
          const int lr = g * kTriL + jj;
          const double y = fma(fb[buf][2][lr], xs[jj + 2], fma(fb[buf][0][lr], xs[jj], fb[buf][1][lr] * xs[jj + 1]));
#pragma unroll
          for (int k = 0; k < NT; ++k) {
            zc[k] = fma(-fb[buf][3 + k][lr], zc[k], y);
            zz[k][jj] = zc[k];
          }
          ax[jj] = a0 * xs[jj + 1] + us[jj];  // + u_1 (phi1 after its first step; else 0)
        }
        chunk_loads(q > 0 ? q - 1 : 0);  // (for q = 0: harmless reads, unused)
#pragma unroll
        for (int jj = kTriL - 1; jj >= 0; --jj) {
          const int lr = g * kTriL + jj;
          const double sp = fb[buf][2][lr];
          double o = ax[jj];
#pragma unroll
          for (int k = 0; k < NT; ++k) {
            // rows past d (tail of the last chunk) leave the carry alone, so
            // the last real row sees x_d = 0
            const double nx = (zz[k][jj] - sk[k] * sp * xc[k]) * fb[buf][3 + kTriTerms + k][lr];
            xc[k] = jj < len ? nx : xc[k];
            o = fma(wk[k], xc[k], o);
          }
          // rows past d store to row r0, which row jj = 0 rewrites last
          const int64_t r = jj < len ? r0 + jj : r0;
          o = first_phi ? o / rN : o;
          gst(dst + r * ldd, o);
          if (first_phi && N > 1) gst(u1 + r * p + c, o);
        }
      }
      if (b > 0) {
        fetch(b - 1);
        put((b - 1) & 1);
        __syncthreads();
      }
    }
    // block 0 is staged in buffer 0 again for the next step's pass 1
  }
}

__global__ void __launch_bounds__(256)
tri_info_kernel(const TriDesc *__restrict__ desc, const PlanRec *__restrict__ plan, InfoRec *__restrict__ info,
                int batch, int order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const PlanRec P = plan[i];
  InfoRec r;
  r.status = P.status;
  r.plan = P.s;
  r.order = order;
  r.ir_iters = 0;
  r.bad_shift = P.bad_shift == 0x7fffffff ? -1 : P.bad_shift;
  r.route = P.route;
  r.norm1 = P.eta;
  r.theta = desc[i].theta;
  r.resid = 0.0;
  info[i] = r;
}

}  // namespace pfm
