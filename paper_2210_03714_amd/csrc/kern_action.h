// Action on a block of vectors: f(A) V by the N-step recurrence of §1.
//
// B = A / N.  One step applies the rational approximant to the current block,
//   r(B) u = a0 u + sum_k w_k (I - c_k B)^{-1} (B u)     (round-off form, §4.3)
// i.e. one product Y = B u and then, for every shift, the solve with the
// factors of I - c_k B computed once for all N steps (§5.1, first remark:
// the LU factorisation is done only once).
// With the hybrid set of §4.3 (exp only) the step adds d1 Y + d2 B Y, a
// second product with the same B.
//   exp:   u_0 = V, u_j = r(B) u_{j-1}, j = 1..N          -> e^A V
//   phi1:  u_1 = (a0' V + sum_k w'_k Z_k(V)) / N,
//          u_{j+1} = r(B) u_j + u_1                       -> phi1(A) V
// (phi1 from the solution u(1) of u' = A u + V, u(0) = 0, the linear ODE of
// §1, stepped with h = 1/N.)
//
// The columns of V are independent, so one workgroup owns one column slab of
// one instance and runs all N steps without talking to any other workgroup.
// The state u lives in registers as MFMA C fragments; B u is a GEMM with B
// (stored column-major by prep_bt_kernel) as the A operand and u staged in LDS
// as the B operand; the row permutation of each factorisation is applied by
// gathering rows of B u from the same LDS buffer.
#pragma once
#include "kern_solve.h"

namespace pfm {

// B column-major npad x npad, zero padded.  action != 0: B = A / N into the
// instance's (otherwise unused) squaring buffer; action == 0: B = A 2^-s into
// the e_off buffer (residual products of the mixed path).
// Grid: x = 32x32 tile, y = instance.
__global__ void __launch_bounds__(256)
prep_bt_kernel(const InstDesc *__restrict__ inst, const PlanRec *__restrict__ plan,
               double *__restrict__ wsd, int action) {
  __shared__ double tile[32][33];
  const int ii = blockIdx.y;
  const InstDesc D = inst[ii];
  const int n = D.n, np = D.npad;
  const int tn = (np + 31) / 32;
  const int tix = blockIdx.x;
  if (tix >= tn * tn) return;
  const int r0 = (tix % tn) * 32, c0 = (tix / tn) * 32;
  const double Nd = (double)plan[ii].s;
  double *Bt = wsd + (action ? D.r_off : D.e_off);
  const int t = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {  // row-major read
    const int r = r0 + (t >> 3), c = c0 + (t & 7) * 4 + u;
    double a = 0.0;
    if (r < n && c < n) {
      a = D.A[(int64_t)r * D.lda + c];
      a = action ? a / Nd : ldexp(a, -plan[ii].s);
    }
    tile[t >> 3][(t & 7) * 4 + u] = a;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {  // column-major write
    const int c = c0 + (t >> 3), r = r0 + (t & 7) * 4 + u;
    if (r < np && c < np) Bt[r + (int64_t)c * np] = tile[(t & 7) * 4 + u][t >> 3];
  }
}

template <int NPMAX, int SW, bool PHI>
__global__ void __launch_bounds__(256, (NPMAX > 256 ? 1 : 2))
action_f64_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nlist,
                  int nslab, const PlanRec *__restrict__ plan, Terms T, double *__restrict__ wsd,
                  const int *__restrict__ wsi) {
  constexpr int RB = NPMAX / 64;
  constexpr int CT = SW / 16;
  __shared__ double Ybuf[NPMAX * SW];
  __shared__ double S[2][16 * SW];
  __shared__ double Tst[4][16 * SW];

  int slot, sl;
  xcd_map(blockIdx.x, nslab, slot, sl);
  if (slot >= nlist) return;
  const int ii = ilist[slot];
  if (!on_route(plan[ii], 0)) return;  // not on the pivoting LU route
  const InstDesc D = inst[ii];
  const int n = D.n, np = D.npad, p = D.p;
  if (np > NPMAX || (np & 15) || n > np || n < 1) return;  // sizes the host never sends
  const int c0 = sl * SW;
  if (c0 >= p) return;
  const int nblk = np >> 4;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  const int N = plan[ii].s;
  const double Nd = (double)N;
  const double *Bt = wsd + D.r_off;
  const int hn = D.hn, emb = D.emb, cin = D.cin;

  v4d u[RB][CT], acc[RB][CT], Z[RB][CT];
  v4d u1[PHI ? RB : 1][CT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int b = wave + 4 * rb;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int col = c0 + 16 * ct + i16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * b + 4 * g + v;
        double x = 0.0;
        if (b < nblk && r < n && col < p) {
          if (!emb)
            x = D.V[(int64_t)r * D.ldv + col];
          else if (r < hn)  // emb(V) first block column: [Re V; Im V]
            x = cin ? D.V[2 * ((int64_t)r * D.ldv + col)] : D.V[(int64_t)r * D.ldv + col];
          else
            x = cin ? D.V[2 * ((int64_t)(r - hn) * D.ldv + col) + 1] : 0.0;
        }
        u[rb][ct][v] = x;
      }
    }
  }

#pragma unroll 1
  for (int step = 0; step < N; ++step) {
    // Y = B u: u to LDS (row-major np x SW), GEMM with B from the workspace
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int b = wave + 4 * rb;
      if (b < nblk) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) Ybuf[(16 * b + 4 * g + v) * SW + 16 * ct + i16] = u[rb][ct][v];
      }
    }
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) Z[rb][ct] = zero4();
#pragma unroll 2
    for (int k0 = 0; k0 < np; k0 += 4) {
      double bf[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) bf[ct] = Ybuf[(k0 + g) * SW + 16 * ct + i16];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int bb = wave + 4 * rb;
        if (bb < nblk) {
          const double a = Bt[(16 * bb + ar) + (int64_t)(k0 + g) * np];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) Z[rb][ct] = mfma16(a, bf[ct], Z[rb][ct]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int b = wave + 4 * rb;
      if (b < nblk) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) Ybuf[(16 * b + 4 * g + v) * SW + 16 * ct + i16] = Z[rb][ct][v];
      }
    }
    __syncthreads();

    // the m shifted solves on P_k^T Y, combined in the round-off form; the
    // hybrid set starts the sum from its polynomial part d1 Y + d2 B Y
    const bool first_phi = PHI && step == 0;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rb][ct] = zero4();
    if (T.d1e != 0.0 || T.d2e != 0.0) {  // (uniform: the call's set)
#pragma unroll 2
      for (int k0 = 0; k0 < np; k0 += 4) {
        double bf[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) bf[ct] = Ybuf[(k0 + g) * SW + 16 * ct + i16];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int bb = wave + 4 * rb;
          if (bb < nblk) {
            const double a = Bt[(16 * bb + ar) + (int64_t)(k0 + g) * np];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[rb][ct] = mfma16(a, bf[ct], acc[rb][ct]);
          }
        }
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[rb][ct][v] = fma(T.d2e, acc[rb][ct][v], T.d1e * Z[rb][ct][v]);
    }
#pragma unroll 1
    for (int k = 0; k < T.nterms; ++k) {
      const int fold = T.fold[k];
      if (fold && T.fn[k] != (first_phi ? 1 : 0)) continue;  // a pair of the other function
      const double w = fold ? 1.0 : (first_phi ? T.wp_re[k] : T.we_re[k]);
      const double fre = fold ? (T.fn[k] ? T.wp_re[k] : T.we_re[k]) : 1.0;
      const double fim = fold ? (T.fn[k] ? T.wp_im[k] : T.we_im[k]) : 0.0;
      if (w == 0.0) continue;
      const double *W = wsd + D.fac_off + (int64_t)k * np * np;
      const int *perm = wsi + D.perm_ioff + (int64_t)k * np;
      const double *dL = wsd + D.dinv_off + (int64_t)(2 * k) * nblk * 256;
      const double *dU = dL + (int64_t)nblk * 256;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int b = wave + 4 * rb;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * b + 4 * g + v;
            double z = 0.0;
            if (b < nblk) {
              const int q = perm[r];
              z = Ybuf[q * SW + 16 * ct + i16];
              if (fold) {  // emb(w Y) = w_re Y + w_im J Y
                const double yj = q < hn ? -Ybuf[(q + hn) * SW + 16 * ct + i16] : Ybuf[(q - hn) * SW + 16 * ct + i16];
                z = fre * z + fim * yj;
              }
            }
            Z[rb][ct][v] = z;
          }
      }
      lu_solve_slab<RB, CT, SW, double>(Z, W, dL, dU, S, Tst[wave], np, nblk, wave, ar, g, i16);
      const double fsc = (fold && T.pair_real) ? 2.0 : 1.0;
      const int frows = (fold && T.pair_real) ? hn : np;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const int r0 = 16 * (wave + 4 * rb) + 4 * g;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (r0 + v < frows) acc[rb][ct][v] = fma(fsc * w, Z[rb][ct][v], acc[rb][ct][v]);
        }
    }
    // next state
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (first_phi) {
            const double x = (T.a0p * u[rb][ct][v] + acc[rb][ct][v]) / Nd;
            if constexpr (PHI) u1[rb][ct][v] = x;
            u[rb][ct][v] = x;
          } else {
            double x = T.a0e * u[rb][ct][v] + acc[rb][ct][v];
            if constexpr (PHI) x += u1[rb][ct][v];
            u[rb][ct][v] = x;
          }
        }
    __syncthreads();
  }

  double *F = PHI ? D.Fp : D.Fe;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int b = wave + 4 * rb;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int col = c0 + 16 * ct + i16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * b + 4 * g + v;
        if (b < nblk && r < n && col < p) {
          if (!emb)
            F[(int64_t)r * D.ldf + col] = u[rb][ct][v];
          else if (cin)
            F[2 * ((int64_t)(r < hn ? r : r - hn) * D.ldf + col) + (r < hn ? 0 : 1)] = u[rb][ct][v];
          else if (r < hn)
            F[(int64_t)r * D.ldf + col] = u[rb][ct][v];
        }
      }
    }
  }
}

}  // namespace pfm
