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
// Two step kernels share the factorisation:
//   tri_scan_kernel (d <= kTsMaxD): a wave per column, 16 rows per lane, the
//     sweeps as affine maps scanned over the lanes; the vector stays in
//     registers for all N steps (described above the kernel);
//   tri_steps_kernel (larger d): a lane per column, a wave per 64 columns of
//     one instance (every factor read is the same address in all lanes), the
//     vector in memory between the passes of a step (below).
// Workspace layout:
//   B:        sub[r] = B[r][r-1] (sub[0] = 0), dia[r], sup[r] = B[r][r+1]
//             (sup[d-1] = 0)
//   factors:  per shift k, l[r] = M[r][r-1] (1 / u[r-1]) (l[0] = 0),
//             ui[r] = 1 / u[r] and em[r] = M[r][r+1] / u[r] (em[d-1] = 0),
//             M = I - c_k B = L U; the backward sweep is then
//             x_r = ui[r] z_r - em[r] x_{r+1}
//   tri_steps_kernel only:
//   vectors:  per function slot, two ping-pong buffers and u_1 (phi1), each
//             d x p row-major (lanes read consecutive addresses)
//   checkpoints: the forward sweep's value at the end of every kTriL-row
//             chunk, per shift, [chunk][k][column]
// A tri_steps_kernel step reads the input vector twice and writes the output
// once: the first pass runs the forward sweeps of all shifts and keeps only
// the chunk-end values; the second pass walks the chunks from the last,
// recomputes each chunk's forward values from its checkpoint in registers,
// and runs the backward sweep, accumulating a0 x + sum_k w_k x_k on the way.
#pragma once
#include <type_traits>

#include "kern_common.h"

namespace pfm {

constexpr int kTriL = 8;         // rows per checkpoint chunk
constexpr int kTriTerms = 10;    // most shifts in a real set (the hybrid set of §4.3)
constexpr int kTsR = 16;         // tri_scan_kernel: rows per lane
constexpr int kTsMaxD = 64 * kTsR;  // its largest d (one wave holds a column)
constexpr int kTsW = 8;          // its waves (columns) per workgroup
constexpr int kFacPF = 16;       // factor kernels: rows whose loads are issued together
static_assert(kFacPF == 16, "tri_factor_kernel stores 4 runs of 16 rows per wave instruction");

struct TriDesc {
  const double *dl, *dd, *du, *V;
  double *Fe, *Fp;
  int64_t ldv, ldf;
  int32_t d, p;
  double theta;
  int64_t b_off;  // sub, dia, sup: 3 d
  int64_t f_off;  // factors: [k][l, ui, em][d]
  int64_t v_off;  // vectors: [slot][3][d][p]
  int64_t c_off;  // checkpoints: [slot][chunk][k][p]
  int32_t wave0;   // first wave of this instance in tri_steps_kernel's launch
  int32_t nwaves;  // its waves: functions x ceil(p / 64) (0: tri_scan_kernel takes it)
  int32_t sg0;     // first workgroup of this instance in tri_scan_kernel's launch
  int32_t nsg;     // its workgroups: functions x ceil(p / kTsW) (0: tri_steps_kernel takes it)
};

struct TriTerms {
  int32_t nterms, nf;
  int32_t fn[2];  // function of each slot: 0 exp, 1 phi1
  double a0e, a0p;
  double c[kTriTerms], we[kTriTerms], wp[kTriTerms];
  double d1, d2;  // the hybrid set's polynomial part d1 x + d2 x^2 (else 0)
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
  // more than kNCap steps: PFM_NOT_COMPUTED, the instance is skipped (the
  // host never reads the plans back, so the cap is applied here)
  if (P.s > kNCap) P.status |= 8;
  plan[ii] = P;
}

// B = A / N and the LU of I - c_k B for every (instance, shift): one thread
// each, a sequential sweep down the diagonal.  A zero or non-finite pivot
// sets PFM_SINGULAR_SHIFT with the smallest such shift.
// One thread per (instance, shift) leaves the chip's SIMDs mostly empty, so
// A's rows are loaded kFacPF at a time from clamped (in-bounds) addresses and
// waited for once per block.  The workgroup is one wave; its 64 threads write
// their factor rows of a block to LDS, and the wave then stores them as runs
// of kFacPF consecutive rows (one thread's l, 1/u or em), so that a store
// instruction touches a few cache lines instead of 64.
__global__ void __launch_bounds__(64)
tri_factor_kernel(const TriDesc *__restrict__ desc, PlanRec *__restrict__ plan, int batch, TriTerms T,
                  double *__restrict__ wsd) {
  __shared__ double buf[3][64][kFacPF + 1];  // a block's l, 1/u, em of each thread
  __shared__ double *dst[3][64];             // where each thread's rows go
  __shared__ int dlen[64];                   // its d (0: nothing to store)
  const int t = threadIdx.x;
  const int gid = blockIdx.x * 64 + t;
  const int ii = gid / T.nterms, k = gid - ii * T.nterms;
  // PFM_NOT_COMPUTED (too many steps) and the grid's padding: no rows
  const bool active = ii < batch && !(plan[ii].status & 8);
  TriDesc D{};
  if (active) D = desc[ii];
  const int d = active ? D.d : 0;
  const double Nd = active ? (double)plan[ii].s : 1.0;
  const double c = T.c[k];
  double *__restrict__ sub = wsd + D.b_off, *__restrict__ dia = sub + d, *__restrict__ sup = dia + d;
  double *__restrict__ l = wsd + D.f_off + (int64_t)k * 3 * d, *__restrict__ ui = l + d, *__restrict__ em = ui + d;
  const double *__restrict__ Al = D.dl, *__restrict__ Ad = D.dd, *__restrict__ Au = D.du;
  dst[0][t] = l;
  dst[1][t] = ui;
  dst[2][t] = em;
  dlen[t] = d;
  const int nt = T.nterms;
  // the instance's shifts share the writing of B (the off-diagonals exist
  // only for d >= 2)
  for (int r0 = k; r0 < d; r0 += kFacPF * nt) {
    double vl[kFacPF], vd[kFacPF], vu[kFacPF];
#pragma unroll
    for (int q = 0; q < kFacPF; ++q) {
      const int r = min(r0 + q * nt, d - 1);
      vd[q] = Ad[r];
      vl[q] = d > 1 ? Al[max(r - 1, 0)] : 0.0;
      vu[q] = d > 1 ? Au[min(r, d - 2)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kFacPF; ++q) {
      const int r = r0 + q * nt;
      const double bs = r > 0 ? vl[q] / Nd : 0.0, bd = vd[q] / Nd, bu = r + 1 < d ? vu[q] / Nd : 0.0;
      if (r < d) {
        sub[r] = bs;
        dia[r] = bd;
        sup[r] = bu;
      }
    }
  }
  bool bad = false;
  double u = 1.0, uinv = 1.0;
  if (d > 0) {
    u = 1.0 - c * (Ad[0] / Nd);
    uinv = 1.0 / u;
    bad |= !(u != 0.0 && isfinite(u));
    l[0] = 0.0;
    ui[0] = uinv;
  }
  int dmax = d;  // the wave's largest d: the blocks below are uniform over the wave
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o));
  // A's rows of a block, read one block ahead through global (not flat)
  // loads, which the LDS accesses of the stores do not have to wait for
  typedef const __attribute__((address_space(1))) double gdouble;
  double al[kFacPF], au[kFacPF], ad[kFacPF];
  auto load_rows = [&](int r0) {
    if (r0 < d) {
#pragma unroll
      for (int q = 0; q < kFacPF; ++q) {
        const int r = min(r0 + q, d - 1);  // >= 1
        al[q] = ((gdouble *)Al)[r - 1];
        au[q] = ((gdouble *)Au)[r - 1];
        ad[q] = ((gdouble *)Ad)[r];
      }
    }
  };
  load_rows(1);
  for (int r0 = 1; r0 < dmax; r0 += kFacPF) {
    double cl[kFacPF], cu[kFacPF], cd[kFacPF];
#pragma unroll
    for (int q = 0; q < kFacPF; ++q) {
      cl[q] = al[q];
      cu[q] = au[q];
      cd[q] = ad[q];
    }
    load_rows(r0 + kFacPF);
    if (r0 < d) {
#pragma unroll
      for (int q = 0; q < kFacPF; ++q) {
        const int r = r0 + q;
        const double mlo = -c * (cl[q] / Nd);  // M[r][r-1]
        const double mup = -c * (cu[q] / Nd);  // M[r-1][r]
        const double lr = mlo * uinv;  // tri_scan_kernel forms the same product from ui
        const double emr = mup * uinv;
        const double un = (1.0 - c * (cd[q] / Nd)) - lr * mup;
        const double unv = 1.0 / un;
        if (r < d) {
          u = un;
          uinv = unv;
          bad |= !(u != 0.0 && isfinite(u));
        }
        buf[0][t][q] = lr;     // l[r]
        buf[1][t][q] = uinv;   // ui[r]
        buf[2][t][q] = emr;    // em[r - 1]
      }
    }
    __syncthreads();
    // run ru = (field, thread): 16 lanes store its rows r0 .. r0 + 15
#pragma unroll 4
    for (int it = 0; it < 3 * kFacPF; ++it) {
      const int ru = it * 4 + (t >> 4), e = t & 15;
      const int f = ru >> 6, tp = ru & 63;
      const int r = r0 + e;
      if (r < dlen[tp]) dst[f][tp][r - (f == 2)] = buf[f][tp][e];
    }
    __syncthreads();  // the next block overwrites buf
  }
  if (d > 0) em[d - 1] = 0.0;
  if (bad) {
    atomicOr(&plan[ii].status, 1);
    atomicMin(&plan[ii].bad_shift, k);
  }
}

// All N steps of one column (lane) of one function slot; one wave per
// workgroup, 64 consecutive columns of one instance.  The instance's B and
// factor rows are staged through LDS in blocks of kTriRB rows (each lane
// loads one row into registers at the start of a block, and writes it into
// the buffer not being read at the block's end); the sweeps read them as
// broadcasts.  The column's own values are read ahead through rings of
// register slots: a ring of kTriFR chunks of x in the forward pass and of
// kTriBR chunk operand sets in the backward pass.  Every chunk of a block is
// unrolled, so a chunk's slot is fixed at compile time and a slot is
// refilled as soon as it has been read: no register move has to wait for a
// load in flight.  fac is the read-only view of B and the factors; vws holds
// the vectors and checkpoints (disjoint parts of the same workspace).  Lanes
// past p repeat column p - 1 and so store what that lane stores.
constexpr int kTriRB = 64;               // rows per staged block (one per lane)
constexpr int kTriCB = kTriRB / kTriL;   // chunks per block
constexpr int kTriFR = 4;                // forward pass: chunks of x in flight
constexpr int kTriBR = 2;                // backward pass: chunk operand sets in flight
static_assert(kTriCB % kTriFR == 0 && kTriCB % kTriBR == 0, "ring sizes divide the chunks of a block");

// Vector loads through global (not flat) instructions: flat
// accesses also count against the LDS counter, so every wait for an LDS read
// would wait for the in-flight prefetches as well.
__device__ __forceinline__ double gld(const double *a) {
  return *(const __attribute__((address_space(1))) double *)a;
}
// The same for this lane's element of a row whose address is wave-uniform:
// the row address (scalar registers; it includes the wave's first column)
// plus the lane's byte offset (a vector register, below 512) is the saddr
// form of the global instructions, so the only address arithmetic left is
// scalar, one add per row.  A row outside the vector reads kTriZeroRow.
__device__ __forceinline__ double gldr(const void *row, uint32_t off) {
  return *(const __attribute__((address_space(1))) double *)((const char *)row + off);
}
__device__ __forceinline__ void gstr(void *row, uint32_t off, double v) {
  *(__attribute__((address_space(1))) double *)((char *)row + off) = v;
}
__device__ double kTriZeroRow[64];        // zero-initialised, never written

// NT: the number of shifts (4, 5, 8, or 10 for the hybrid set), so that the
// sweeps of all shifts unroll without branches and their chains interleave.
// PHI: some slot of the launch is phi1, whose steps after the first add u_1
// (without it, no u_1 row is read).  HYB: the hybrid set of §4.3 (exp only;
// R10' of §5 on a tridiagonal A): the forward pass also forms
// P = d1 B y + d2 B (B y) for y = x, one row behind, into the slot's u_1
// buffer, and the backward pass adds it where phi1 adds u_1.  The backward sweeps run in two halves of the shifts
// (all of them for NT = 4), so that only half of the recomputed forward
// values are held at a time; the sum a0 x + sum_k w_k x_k keeps the order
// k = 0, 1, ...  Chunks that start past d are skipped; the tail rows of the
// last chunk are swept on zero factors and never stored.
template <int NT, bool PHI, bool HYB>
__global__ void __launch_bounds__(64)
tri_steps_kernel(const TriDesc *__restrict__ desc, int batch, const PlanRec *__restrict__ plan, TriTerms T,
                 const double *__restrict__ fac, double *__restrict__ vws) {
  constexpr int KF = 3 + 3 * NT;  // staged fields: sub, dia, sup, then l_k, ui_k, em_k
  constexpr bool ADD = PHI || HYB;  // the backward pass adds a stored row (u_1 or P)
  __shared__ double fb[2][KF][kTriRB];
  constexpr int NA = NT > 4 ? (NT + 1) / 2 : NT;  // shifts of the first half
  const int lane = threadIdx.x;
  const int gw = blockIdx.x;
  int lo = 0, hi = batch - 1;  // the instance whose waves contain gw
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].wave0 <= gw) lo = mid;
    else hi = mid - 1;
  }
  const int ii = __builtin_amdgcn_readfirstlane(lo);
  if (plan[ii].status & 8) return;  // PFM_NOT_COMPUTED: the whole wave leaves before any barrier
  const TriDesc D = desc[ii];
  const int d = D.d, p = D.p;
  const int cpw = (p + 63) / 64;
  const int wl = gw - D.wave0;
  const int slot = wl / cpw;
  const int cb = (wl - slot * cpw) * 64;  // the wave's first column
  // lanes past p repeat column p - 1 exactly (same inputs, same arithmetic),
  // so their stores write the values that lane writes: no store needs a mask
  const int c = cb + lane < p ? cb + lane : p - 1;
  const int fn = slot == 0 ? T.fn[0] : T.fn[1];
  const int N = plan[ii].s;
  const int nch = (d + kTriL - 1) / kTriL;
  const int nb = (d + kTriRB - 1) / kTriRB;
  const double *sub = fac + D.b_off, *dia = sub + d, *sup = dia + d;
  const double *lf = fac + D.f_off;
  const int64_t dp = (int64_t)d * p;
  double *vb = vws + D.v_off + (int64_t)slot * 3 * dp;
  double *u1 = vb + 2 * dp;
  char *ckb = (char *)(vws + D.c_off + (int64_t)slot * nch * NT * p + cb);
  char *u1b = (char *)(u1 + cb);
  const char *zrow = (const char *)kTriZeroRow;
  const uint32_t cofs = 8u * (uint32_t)(c - cb);  // this lane's byte offset from column cb
  const int64_t p8 = 8 * (int64_t)p;

  double nf[KF];
  // rows past d are staged as zeros (read from sub[0]): there y = 0, z = 0
  // and x = 0, so the last real row sees x_d = 0 with no test in the sweeps
  auto fetch = [&](int blk) {
    const int r = blk * kTriRB + lane;
    const bool in = r < d;
    nf[0] = gld(in ? sub + r : sub);
    nf[1] = gld(in ? dia + r : sub);
    nf[2] = gld(in ? sup + r : sub);
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const double *a = lf + (int64_t)k * 3 * d + r;
      nf[3 + k] = gld(in ? a : sub);
      nf[3 + NT + k] = gld(in ? a + d : sub);
      nf[3 + 2 * NT + k] = gld(in ? a + 2 * d : sub);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int f = 0; f < KF; ++f) fb[buf][f][lane] = nf[f];
  };
  fetch(0);
  put(0);
  __syncthreads();

#pragma unroll 1
  for (int j = 0; j < N; ++j) {
    const char *srcb = (const char *)((j == 0 ? D.V : vb + (int64_t)((j - 1) & 1) * dp) + cb);
    const int64_t lds8 = 8 * (j == 0 ? D.ldv : (int64_t)p);
    char *dstb = (char *)((j == N - 1 ? (fn ? D.Fp : D.Fe) : vb + (int64_t)(j & 1) * dp) + cb);
    const int64_t ldd8 = 8 * (j == N - 1 ? D.ldf : (int64_t)p);
    // phi1's first step is u_1 = rho(B) V / N: the 1/N is folded into its
    // weights
    const bool first_phi = fn == 1 && j == 0;
    const double a0 = first_phi ? T.a0p / (double)N : T.a0e;
    // cnt consecutive rows of x from row r (rows outside [0, d) read the
    // zero row: the address is chosen, not the value, so no load sits behind
    // a branch)
    auto xrows = [&](int r, double *out, auto cntc) {
      const char *rp = srcb + (int64_t)r * lds8;
#pragma unroll
      for (int jj = 0; jj < decltype(cntc)::value; ++jj, rp += lds8) {
        const bool ok = r + jj >= 0 && r + jj < d;
        out[jj] = gldr(ok ? rp : zrow, cofs);
      }
    };
    using Lc = std::integral_constant<int, kTriL>;

    // pass 1 (block 0 is staged in buffer 0): forward sweeps
    // z_r = y_r - l_r z_{r-1} of every shift, y = B x; keep z at the end of
    // each chunk.  Chunk g's rows sit in ring slot g mod kTriFR; the slot is
    // refilled with the rows kTriFR chunks further down once it is read.
    {
      double z[NT];
#pragma unroll
      for (int k = 0; k < NT; ++k) z[k] = 0.0;
      double xm = 0.0, xr[kTriFR][kTriL];
#pragma unroll
      for (int i = 0; i < kTriFR; ++i) xrows(i * kTriL, xr[i], Lc());
      // HYB: y and B's row of the two rows before the current one
      double ym1 = 0.0, ym2 = 0.0, bs1 = 0.0, bd1 = 0.0, bu1 = 0.0;
#pragma unroll 1
      for (int b = 0; b < nb; ++b) {
        const int buf = b & 1;
        fetch(b + 1 < nb ? b + 1 : b);  // staged at the end of this block
#pragma unroll
        for (int g = 0; g < kTriCB; ++g) {
          const int rg = b * kTriRB + g * kTriL;
          const int sl = g % kTriFR, sn = (g + 1) % kTriFR;
          if (rg < d) {
#pragma unroll
            for (int jj = 0; jj < kTriL; ++jj) {
              const int lr = g * kTriL + jj;
              const double x0 = xr[sl][jj];
              const double xp = jj + 1 < kTriL ? xr[sl][jj + 1] : xr[sn][0];
              const double y = fma(fb[buf][2][lr], xp, fma(fb[buf][0][lr], xm, fb[buf][1][lr] * x0));
#pragma unroll
              for (int k = 0; k < NT; ++k) z[k] = fma(-fb[buf][3 + k][lr], z[k], y);
              xm = x0;
              if constexpr (HYB) {
                // P on the row before: d1 y + d2 (B y), whose last term needs
                // this row's y (rows past d have y = 0)
                const int r = rg + jj;
                const double by = fma(bu1, y, fma(bs1, ym2, bd1 * ym1));
                const double pv = fma(T.d2, by, T.d1 * ym1);
                if (r >= 1 && r - 1 < d) gstr(u1b + (int64_t)(r - 1) * p8, cofs, pv);
                ym2 = ym1;
                ym1 = y;
                bs1 = fb[buf][0][lr];
                bd1 = fb[buf][1][lr];
                bu1 = fb[buf][2][lr];
              }
            }
            // (the last chunk's slot is written and never read)
            char *cq = ckb + (int64_t)(rg / kTriL) * NT * p8;
#pragma unroll
            for (int k = 0; k < NT; ++k, cq += p8) gstr(cq, cofs, z[k]);
          }
          xrows(rg + kTriFR * kTriL, xr[sl], Lc());
        }
        if (b + 1 < nb) {
          put(buf ^ 1);
          __syncthreads();
        }
      }
      if constexpr (HYB) {
        // d a multiple of kTriL: no row past d was swept, and P on the last
        // row (whose B y has no row below) is still due
        if (d % kTriL == 0) {
          const double by = fma(bs1, ym2, bd1 * ym1);
          gstr(u1b + (int64_t)(d - 1) * p8, cofs, fma(T.d2, by, T.d1 * ym1));
        }
      }
    }

    // pass 2 (block nb - 1 is staged): chunks from the last.  Per chunk q
    // (ring slot q mod kTriBR): y = B x on its rows, then for each half of
    // the shifts the forward values from the chunk's checkpoints and the
    // backward sweeps x_r = ui_r z_r - em_r x_{r+1}, the shifts of the half
    // row by row
    // (independent chains side by side), and out_r = a0 x_r + sum_k w_k x_{k,r}.
    // Once the slot is read, it is refilled with chunk q - kTriBR.
    {
      const bool add_u1 = (PHI && fn == 1 && j > 0) || HYB;
      double xs[kTriBR][kTriL + 1];            // rows r0 - 1 .. r0 + kTriL - 1
      double us[kTriBR][ADD ? kTriL : 1];      // u_1 (or P) on the chunk's rows
      double zc[kTriBR][NT];                   // checkpoints: z at row r0 - 1
      auto chunk_loads = [&](int q, int sl) {
        xrows(q * kTriL - 1, xs[sl], std::integral_constant<int, kTriL + 1>());
        if constexpr (ADD) {
          const char *up = u1b + (int64_t)q * kTriL * p8;
#pragma unroll
          for (int jj = 0; jj < kTriL; ++jj, up += p8) {
            const int r = q * kTriL + jj;
            const bool ok = add_u1 && r >= 0 && r < d;
            us[sl][jj] = gldr(ok ? up : zrow, cofs);
          }
        }
        const bool okc = q > 0 && q < nch;
        const char *cp = ckb + (int64_t)(q - 1) * NT * p8;
#pragma unroll
        for (int k = 0; k < NT; ++k, cp += p8) zc[sl][k] = gldr(okc ? cp : zrow, cofs);
      };
      double xc[NT], wk[NT];
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        xc[k] = 0.0;
        wk[k] = first_phi ? T.wp[k] / (double)N : T.we[k];
      }
      const int qtop = nb * kTriCB - 1;  // the last block's last chunk
#pragma unroll
      for (int i = 0; i < kTriBR; ++i) chunk_loads(qtop - i, (kTriCB - 1 - i) % kTriBR);
      double xt = 0.0;  // x on row r0 + kTriL (0 past the last row)
#pragma unroll 1
      for (int b = nb - 1; b >= 0; --b) {
        const int buf = b & 1;
        fetch(b > 0 ? b - 1 : 0);  // staged at the end of this block
#pragma unroll
        for (int g = kTriCB - 1; g >= 0; --g) {
          const int sl = g % kTriBR;
          const int q = b * kTriCB + g;
          const int r0 = q * kTriL;
          const bool live = r0 < d;
          const int len = d - r0 < kTriL ? d - r0 : kTriL;
          double y[kTriL], o[kTriL];
          // one half of the shifts, [K0, K1): forward values from the
          // checkpoints, then (when SWEEP) the backward sweeps into o
          auto recompute = [&](auto k0c, auto k1c, double (*zz)[kTriL]) {
            constexpr int K0 = decltype(k0c)::value, K1 = decltype(k1c)::value;
#pragma unroll
            for (int jj = 0; jj < kTriL; ++jj) {
              const int lr = g * kTriL + jj;
#pragma unroll
              for (int k = K0; k < K1; ++k) {
                zc[sl][k] = fma(-fb[buf][3 + k][lr], zc[sl][k], y[jj]);
                zz[k - K0][jj] = zc[sl][k];
              }
            }
          };
          auto sweep = [&](auto k0c, auto k1c, double (*zz)[kTriL]) {
            constexpr int K0 = decltype(k0c)::value, K1 = decltype(k1c)::value;
#pragma unroll
            for (int jj = kTriL - 1; jj >= 0; --jj) {
              const int lr = g * kTriL + jj;
#pragma unroll
              for (int k = K0; k < K1; ++k) {
                xc[k] = fma(-fb[buf][3 + 2 * NT + k][lr], xc[k], fb[buf][3 + NT + k][lr] * zz[k - K0][jj]);
                o[jj] = fma(wk[k], xc[k], o[jj]);
              }
            }
          };
          double za[NA][kTriL];
          double zb[NT - NA > 0 ? NT - NA : 1][kTriL];
          if (live) {
#pragma unroll
            for (int jj = 0; jj < kTriL; ++jj) {
              const int lr = g * kTriL + jj;
              const double xh = jj + 1 < kTriL ? xs[sl][jj + 2] : xt;
              y[jj] = fma(fb[buf][2][lr], xh, fma(fb[buf][0][lr], xs[sl][jj], fb[buf][1][lr] * xs[sl][jj + 1]));
              double ax = a0 * xs[sl][jj + 1];
              if constexpr (ADD) ax += us[sl][jj];  // u_1 (phi1 after its first step) or P; else 0
              o[jj] = ax;
            }
            xt = xs[sl][1];
            recompute(std::integral_constant<int, 0>(), std::integral_constant<int, NA>(), za);
            sweep(std::integral_constant<int, 0>(), std::integral_constant<int, NA>(), za);
            if constexpr (NT > NA)
              recompute(std::integral_constant<int, NA>(), std::integral_constant<int, NT>(), zb);
          }
          chunk_loads(q - kTriBR, sl);  // (chunks below 0 read harmless addresses, unused)
          if (live) {
            if constexpr (NT > NA) sweep(std::integral_constant<int, NA>(), std::integral_constant<int, NT>(), zb);
#pragma unroll
            for (int jj = kTriL - 1; jj >= 0; --jj) {
              // rows past d store to row r0, which row jj = 0 rewrites last
              const int64_t r = jj < len ? r0 + jj : r0;
              gstr(dstb + r * ldd8, cofs, o[jj]);
              if (first_phi && N > 1) gstr(u1b + r * p8, cofs, o[jj]);
            }
          }
        }
        if (b > 0) {
          put((b - 1) & 1);
          __syncthreads();
        }
      }
    }
    // block 0 is staged in buffer 0 again for the next step's pass 1
  }
}

// One double through a DPP lane move (two 32-bit moves).  Lanes whose source
// lies outside the pattern, and rows that RM leaves out, take `old`.
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ double dpp_f64(double src, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(src), CTRL, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(src), CTRL, RM, 0xf, false);
  return __hiloint2double(hi, lo);
}
// A double moved by the DPP pattern CTRL, 0 in the lanes with no source lane
// (bound control set), so no old value has to be written first.
template <int CTRL>
__device__ __forceinline__ double dpp0_f64(double src) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(src), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(src), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// The value entering lane L of the recurrence Z_L = g_L Z_{L-1} + h_L,
// Z_{-1} = 0 (lane 0 gets 0): an inclusive scan of the maps (g, h) over the
// wave, composed as (g, h) after (g', h') = (g g', g h' + h): shifts by 1, 2,
// 4, 8 within each row of 16 lanes, then row 0's total into row 1 and row
// 2's into row 3, then rows 0-1's into rows 2 and 3; the result moved up one
// lane.  Lanes left without a source compose with the identity (1, 0).
__device__ __forceinline__ double scan_in_fwd(double g, double h, int lane) {
#define PFM_SCAN_LEVEL(CTRL, RM)                        \
  {                                                     \
    const double gp = dpp_f64<CTRL, RM>(g, 1.0);        \
    const double hp = dpp_f64<CTRL, RM>(h, 0.0);        \
    h = fma(g, hp, h);                                  \
    g *= gp;                                            \
  }
  PFM_SCAN_LEVEL(0x111, 0xf)  // row_shr:1
  PFM_SCAN_LEVEL(0x112, 0xf)  // row_shr:2
  PFM_SCAN_LEVEL(0x114, 0xf)  // row_shr:4
  PFM_SCAN_LEVEL(0x118, 0xf)  // row_shr:8
  PFM_SCAN_LEVEL(0x142, 0xa)  // row_bcast:15 into rows 1 and 3
  PFM_SCAN_LEVEL(0x143, 0xc)  // row_bcast:31 into rows 2 and 3
#undef PFM_SCAN_LEVEL
  (void)lane;
  return dpp_f64<0x138>(h, 0.0);  // wave_shr:1
}

// The value entering lane L of X_L = G_L X_{L+1} + H_L, X_64 = 0 (lane 63
// gets 0): shifts by 1, 2, 4, 8 towards lane 0 within each row, then each
// row's map is applied to the value leaving the rows above it (the row
// totals sit in lanes 16, 32, 48; wave-uniform), then moved down one lane.
__device__ __forceinline__ double scan_in_bwd(double G, double H, int lane) {
#define PFM_SCAN_LEVEL(CTRL)                          \
  {                                                   \
    const double Gp = dpp_f64<CTRL>(G, 1.0);          \
    const double Hp = dpp_f64<CTRL>(H, 0.0);          \
    H = fma(G, Hp, H);                                \
    G *= Gp;                                          \
  }
  PFM_SCAN_LEVEL(0x101)  // row_shl:1
  PFM_SCAN_LEVEL(0x102)  // row_shl:2
  PFM_SCAN_LEVEL(0x104)  // row_shl:4
  PFM_SCAN_LEVEL(0x108)  // row_shl:8
#undef PFM_SCAN_LEVEL
  const double s2 = readlane_f64(H, 48);                          // leaving row 2 upwards: row 3's total on 0
  const double s1 = fma(readlane_f64(G, 32), s2, readlane_f64(H, 32));
  const double s0 = fma(readlane_f64(G, 16), s1, readlane_f64(H, 16));
  const int row = lane >> 4;
  const double sin = row == 0 ? s0 : row == 1 ? s1 : row == 2 ? s2 : 0.0;
  H = fma(G, sin, H);
  return dpp_f64<0x130>(H, 0.0);  // wave_shl:1
}

// The same values when every lane's multiplier is at most 2^-30 in
// magnitude: the value entering lane L is then h_{L-1} + g_{L-1} h_{L-2} up
// to g_{L-1} g_{L-2} Z_{L-3}, below 2^-60 max|Z|, so two lanes' maps carry
// every digit (the planned B makes |l_r|, |em_r| < 0.06, so a lane's
// product of 16 is below 1e-19).
// Lane L - 1 forms h_{L-1} + g_{L-1} h_{L-2} with its own multiplier and one
// move passes it to lane L (lane 0 gets 0).
__device__ __forceinline__ double scan_in_fwd2(double g, double h) {
  return dpp0_f64<0x138>(fma(g, dpp0_f64<0x138>(h), h));  // wave_shr:1
}
__device__ __forceinline__ double scan_in_bwd2(double G, double H) {
  return dpp0_f64<0x130>(fma(G, dpp0_f64<0x130>(H), H));  // wave_shl:1
}

// All N steps of the tridiagonal action with a wave per column: lane L holds
// rows 16 L .. 16 L + 15 of the column, so the vector and every intermediate
// stay in registers for the whole call (d <= kTsMaxD).  The sweeps of each
// shifted system run as affine recurrences split at lane boundaries:
//   forward  z_r = y_r - l_r z_{r-1}:  each lane composes its rows into one
//            map Z_L = g_L Z_{L-1} + h_L, an inclusive scan over the lanes
//            gives every lane the value entering its rows, and the lane then
//            runs its rows again from that value;
//   backward x_r = ui_r z_r - em_r x_{r+1}: the same with the maps composed
//            from the last row up and the scan from lane 63 down.
// A workgroup is kTsW columns of one function slot of one instance; it
// stages the instance's B and 1/u of every shift in LDS once, transposed so
// that the lanes' reads of one row index are consecutive, and forms l and em
// from them as tri_factor_kernel does:
//   l_r = (-c_k B[r][r-1]) ui_{r-1},   -em_r = (c_k B[r][r+1]) ui_r.
// Rows past d are staged as zeros, so they hold y = z = x = 0.  Waves past p
// repeat column p - 1 (same inputs, same arithmetic, same stores).  No
// barrier follows the staging: each wave runs its column to the end.
// NT, PHI and HYB as in tri_steps_kernel.
template <int NT, bool PHI, bool HYB>
__global__ void __launch_bounds__(64 * kTsW)
tri_scan_kernel(const TriDesc *__restrict__ desc, int batch, const PlanRec *__restrict__ plan, TriTerms T,
                const double *__restrict__ fac, int nsg) {
  // LST (up to 8 shifts, where it fits the 160 KiB of LDS): -l_k and ui_k
  // of every shift are staged, and each lane's composed products
  //   g_{k,L} = prod_i (-l_r),  G_{k,L} = prod_i (-em_r)  over its rows r
  // are formed once per workgroup, so that a shift costs 8 FP64 operations
  // per row: the lane's rows are swept from the value entering them, twice
  // per direction.  Otherwise (the 10 shifts of the hybrid set) only ui_k is
  // staged, l and em are formed per row, and the lane's sweeps keep the
  // running products, 10 operations per row.
  constexpr bool LST = NT <= 8;
  constexpr int NF = LST ? 3 + 2 * NT : 3 + NT;  // sub, dia, sup, then (-l_k, ui_k) or ui_k
  constexpr int R = kTsR;
  constexpr int NTAB = LST ? 2 * NT * 64 : 0;  // g then G, [k][lane]
  __shared__ double st[NF * kTsMaxD + NTAB];  // field f, row r at f * kTsMaxD + (r % R) * 64 + r / R
  const int t = threadIdx.x, lane = t & 63;
  // workgroup b runs on XCD b mod 8: XCD x takes the x-th eighth of the
  // workgroups in order, so the workgroups of one instance share an L2
  const int sgw = (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3));
  if (sgw >= nsg) return;  // grid padding: uniform over the workgroup, before the barrier
  int lo = 0, hi = batch - 1;  // the instance whose workgroups contain this one
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].sg0 <= sgw) lo = mid;
    else hi = mid - 1;
  }
  const int ii = lo;
  if (plan[ii].status & 8) return;  // PFM_NOT_COMPUTED: uniform over the workgroup, before the barrier
  const TriDesc D = desc[ii];
  const int d = D.d, p = D.p;
  const int cpg = (p + kTsW - 1) / kTsW;
  const int wl = sgw - D.sg0;
  const int slot = wl / cpg;
  int col = (wl - slot * cpg) * kTsW + (t >> 6);
  if (col >= p) col = p - 1;
  const int fn = slot == 0 ? T.fn[0] : T.fn[1];
  const int N = plan[ii].s;

  {
    const double *bsrc = fac + D.b_off;  // sub, dia, sup: d each
    const double *usrc = fac + D.f_off;  // per shift l, ui, em: d each
    // a thread per (field, lane): the lane's R rows from global memory into
    // registers, then into LDS, where the 64 lanes' writes are consecutive
    for (int q = t; q < NF * 64; q += 64 * kTsW) {
      const int f = q >> 6;  // uniform over the wave
      const double *src;
      double sg = 1.0;
      if (f < 3) src = bsrc + (int64_t)f * d;
      else if (LST) {
        src = usrc + (int64_t)((f - 3) >> 1) * 3 * d + ((f - 3) & 1 ? d : 0);
        if (!((f - 3) & 1)) sg = -1.0;
      } else {
        src = usrc + (int64_t)(f - 3) * 3 * d + d;
      }
      double v[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int r = lane * R + i;
        v[i] = r < d ? sg * src[r] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < R; ++i) st[f * kTsMaxD + i * 64 + lane] = v[i];
    }
  }
  __syncthreads();
  const double *sl = st + lane;  // this lane's rows: sl[f * kTsMaxD + i * 64]
  auto ld = [&](int f, int i) { return sl[f * kTsMaxD + i * 64]; };
  bool short_scan = false;  // every lane product at most 2^-30 (scan_in_fwd2)
  if constexpr (LST) {
    // the lanes' products, one (shift, lane) per thread
    for (int q = t; q < NT * 64; q += 64 * kTsW) {
      const int k = q >> 6, L = q & 63;
      const double *rw = st + L;
      double g = 1.0, G = 1.0;
      for (int i = 0; i < R; ++i) g *= rw[(3 + 2 * k) * kTsMaxD + i * 64];
      for (int i = R - 1; i >= 0; --i)
        G *= (T.c[k] * rw[2 * kTsMaxD + i * 64]) * rw[(4 + 2 * k) * kTsMaxD + i * 64];
      st[NF * kTsMaxD + q] = g;
      st[NF * kTsMaxD + NT * 64 + q] = G;
    }
    __syncthreads();
    // each wave (one column) decides for itself: the same tables, the same vote
    int big = 0;
    for (int k = 0; k < NT; ++k)
      big |= !(fabs(st[NF * kTsMaxD + k * 64 + lane]) <= 0x1p-30 &&
               fabs(st[NF * kTsMaxD + (NT + k) * 64 + lane]) <= 0x1p-30);  // (NaN too)
    short_scan = !__any(big);
  }
  // exp: the lane products of the next shift pair (forward, backward), read
  // one pair ahead so that the scans do not wait for LDS
  double gq[2] = {0.0, 0.0}, Gq[2] = {0.0, 0.0};
  auto load_g = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int kk = min(k0 + j, NT - 1);
      gq[j] = st[NF * kTsMaxD + kk * 64 + lane];
      Gq[j] = st[NF * kTsMaxD + (NT + kk) * 64 + lane];
    }
  };
  if constexpr (LST && !PHI) load_g(0);

  const int r0 = lane * R;
  double y[R];
  {
    const double *vp = D.V + col;
#pragma unroll
    for (int i = 0; i < R; ++i) y[i] = r0 + i < d ? vp[(int64_t)(r0 + i) * D.ldv] : 0.0;
  }
  double u1[PHI ? R : 1];
#pragma unroll 1
  for (int j = 0; j < N; ++j) {
    // phi1's first step is u_1 = rho(B) V / N: the 1/N is folded into its weights
    const bool first_phi = fn == 1 && j == 0;
    const double a0 = first_phi ? T.a0p / (double)N : T.a0e;
    // y <- B y's input; f = B y, acc = a0 y (+ u_1 or P)
    double fv[R], acc[R];
    {
      // the neighbouring lanes' edge rows (0 past the wave's ends), by DPP
      const double yup = dpp0_f64<0x138>(y[R - 1]), ydn = dpp0_f64<0x130>(y[0]);  // wave_shr:1, wave_shl:1
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const double ym = i > 0 ? y[i - 1] : yup, yp = i + 1 < R ? y[i + 1] : ydn;
        fv[i] = fma(ld(2, i), yp, fma(ld(0, i), ym, ld(1, i) * y[i]));
      }
#pragma unroll
      for (int i = 0; i < R; ++i) acc[i] = a0 * y[i];
      if constexpr (PHI) {
        if (fn == 1 && j > 0) {
#pragma unroll
          for (int i = 0; i < R; ++i) acc[i] += u1[i];
        }
      }
      if constexpr (HYB) {
        // P = d1 f + d2 B f (the hybrid set's polynomial part, §4.3)
        const double fup = dpp0_f64<0x138>(fv[R - 1]), fdn = dpp0_f64<0x130>(fv[0]);
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const double fm = i > 0 ? fv[i - 1] : fup, fp = i + 1 < R ? fv[i + 1] : fdn;
          const double bf = fma(ld(2, i), fp, fma(ld(0, i), fm, ld(1, i) * fv[i]));
          acc[i] += fma(T.d2, bf, T.d1 * fv[i]);
        }
      }
    }
    typedef const __attribute__((address_space(3))) double lds_double;
    if constexpr (LST) {
      // KP shifts at a time from k0, their chains side by side; the sum
      // keeps the order k = 0, 1, ...
      auto run_shifts = [&](auto kpc, int k0) {
        constexpr int KP = decltype(kpc)::value;
        double A[KP][R], z[KP][R], ck[KP], wk[KP];
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          ck[j] = T.c[k0 + j];
          wk[j] = first_phi ? T.wp[k0 + j] / (double)N : T.we[k0 + j];
        }
        // B's rows are read again for every shift pair: held across them
        // they would take 64 more registers per lane
        lds_double *sk = (lds_double *)sl;
        asm volatile("" : "+v"(sk));
        auto lk = [&](int f, int i) { return sk[f * kTsMaxD + i * 64]; };
        auto gfw = [&](int j) -> double {
          if constexpr (PHI) return sk[NF * kTsMaxD + (k0 + j) * 64];
          else return gq[j];
        };
        auto gbw = [&](int j) -> double {
          if constexpr (PHI) return sk[NF * kTsMaxD + (NT + k0 + j) * 64];
          else return Gq[j];
        };
        // forward: the lane's rows from a zero start (its map's offset), the
        // scan, then the rows again from the value entering them
        double h[KP], zp[KP];
#pragma unroll
        for (int j = 0; j < KP; ++j) h[j] = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
#pragma unroll
          for (int j = 0; j < KP; ++j) {
            const double nl = lk(3 + 2 * (k0 + j), i);
            A[j][i] = nl;
            h[j] = fma(nl, h[j], fv[i]);
          }
        }
        if (short_scan) {
#pragma unroll
          for (int j = 0; j < KP; ++j) zp[j] = scan_in_fwd2(gfw(j), h[j]);
        } else {
#pragma unroll
          for (int j = 0; j < KP; ++j) zp[j] = scan_in_fwd(gfw(j), h[j], lane);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
#pragma unroll
          for (int j = 0; j < KP; ++j) {
            zp[j] = fma(A[j][i], zp[j], fv[i]);
            z[j][i] = zp[j];
          }
        }
        // backward: z <- ui z, A <- -em, the same in the other direction
#pragma unroll
        for (int j = 0; j < KP; ++j) h[j] = 0.0;
#pragma unroll
        for (int i = R - 1; i >= 0; --i) {
          const double sup = lk(2, i);
#pragma unroll
          for (int j = 0; j < KP; ++j) {
            const double ui = lk(4 + 2 * (k0 + j), i);
            const double e = (ck[j] * sup) * ui;
            const double sv = ui * z[j][i];
            A[j][i] = e;
            z[j][i] = sv;
            h[j] = fma(e, h[j], sv);
          }
        }
        if (short_scan) {
#pragma unroll
          for (int j = 0; j < KP; ++j) zp[j] = scan_in_bwd2(gbw(j), h[j]);
        } else {
#pragma unroll
          for (int j = 0; j < KP; ++j) zp[j] = scan_in_bwd(gbw(j), h[j], lane);
        }
        if constexpr (!PHI) load_g(k0 + KP < NT ? k0 + KP : 0);  // the next pair's (or the next step's first)
#pragma unroll
        for (int i = R - 1; i >= 0; --i) {
#pragma unroll
          for (int j = 0; j < KP; ++j) {
            zp[j] = fma(A[j][i], zp[j], z[j][i]);
            acc[i] = fma(wk[j], zp[j], acc[i]);
          }
        }
      };
#pragma unroll 1
      for (int k = 0; k + 2 <= NT; k += 2) run_shifts(std::integral_constant<int, 2>(), k);
      if constexpr (NT & 1) run_shifts(std::integral_constant<int, 1>(), NT - 1);
    } else {
#pragma unroll 1
      for (int k = 0; k < NT; ++k) {
        const double ck = T.c[k], nck = -ck;
        const double wk = first_phi ? T.wp[k] / (double)N : T.we[k];
        double A[R], z[R];
        // B's rows are read again for every shift: held across the shifts
        // they would take 64 more registers per lane
        lds_double *sk = (lds_double *)sl;
        asm volatile("" : "+v"(sk));
        auto lk = [&](int f, int i) { return sk[f * kTsMaxD + i * 64]; };
        // forward, this lane's rows from a zero start: z0 into z, and the
        // products gamma_i = prod_{i' <= i} (-l_i') into A, so that
        // z_i = z0_i + gamma_i z_in once the value entering the lane is known
        double h = 0.0, g = 1.0;
        double uprev = lane > 0 ? st[(3 + k) * kTsMaxD + (R - 1) * 64 + lane - 1] : 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const double ui = lk(3 + k, i);
          const double l = (nck * lk(0, i)) * uprev;
          h = fma(-l, h, fv[i]);
          g *= -l;
          z[i] = h;
          A[i] = g;
          uprev = ui;
        }
        const double zin = __any(!(fabs(g) <= 0x1p-30)) ? scan_in_fwd(g, h, lane) : scan_in_fwd2(g, h);
#pragma unroll
        for (int i = 0; i < R; ++i) z[i] = fma(A[i], zin, z[i]);
        // backward, from this lane's last row with a zero start: x0 into z,
        // delta_i = prod_{i' >= i} (-em_i') into A; x_i = x0_i + delta_i x_in
        double H = 0.0, G = 1.0;
#pragma unroll
        for (int i = R - 1; i >= 0; --i) {
          const double ui = lk(3 + k, i);
          const double e = (ck * lk(2, i)) * ui;
          H = fma(e, H, ui * z[i]);
          G *= e;
          z[i] = H;
          A[i] = G;
        }
        const double xin = __any(!(fabs(G) <= 0x1p-30)) ? scan_in_bwd(G, H, lane) : scan_in_bwd2(G, H);
#pragma unroll
        for (int i = 0; i < R; ++i) acc[i] = fma(wk, fma(A[i], xin, z[i]), acc[i]);
      }
    }
    if constexpr (PHI) {
      if (first_phi && N > 1) {
#pragma unroll
        for (int i = 0; i < R; ++i) u1[i] = acc[i];
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) y[i] = acc[i];
  }
  {
    double *fp = (fn ? D.Fp : D.Fe) + col;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (r0 + i < d) fp[(int64_t)(r0 + i) * D.ldf] = y[i];
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
