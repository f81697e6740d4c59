// Shifted solves fused with the linear combination (full-matrix path).
//
// For every nonzero shift c_k the paper needs Z_k = (I - c_k B)^{-1} B (the
// round-off form of §4.3: the right-hand side is B, not I), and the result is
//   R   = a0 I + sum_k w_k   Z_k      (exp,  w_k   = b_k   c_k)
//   Phi = a0' I + sum_k w'_k Z_k      (phi1, w'_k  = b'_k  c_k)
// from the same solves (§2: several functions from one set of F_i).
//
// One workgroup owns one column slab (SW columns) of one instance and loops
// over all shifts, accumulating w_k Z_k in registers; no Z_k ever reaches
// memory and the slab of R (and Phi) is written once, column-major, into the
// squaring buffers.
//
// Block substitution without diagonal solves on the critical path: with the
// LU kernel's L'_ij = L_ij inv(L_jj), the forward recurrence
//   Y_i <- Y_i - sum_{j<i} L'_ij Y_j      (Y = P^T B[:, slab] initially)
// runs on un-normalised blocks, and Z_i = inv(L_ii) Y_i afterwards, for all i
// at once (the same algebra as Z_i = inv(L_ii)(Y_i - sum_j L_ij Z_j)).  The
// backward pass with U'_ij = U_ij inv(U_jj) is the mirror image.  Each step is
// then: the owner wave posts its finished block to a double-buffered LDS slab,
// one barrier, and every wave updates its own blocks below (MFMA, A operand
// from the factor buffer, loaded before the barrier).
//
// Register layout: row block b (16 rows) belongs to wave b mod 4; each wave
// holds RB = NPMAX/64 row blocks x CT = SW/16 column tiles of Z and of the
// accumulators as MFMA C fragments.
#pragma once
#include "kern_common.h"

namespace pfm {

// Z[rb] <- inv(D_b) Z[rb] for the row blocks this wave owns (D = L or U
// diagonal blocks, stored inverted, column-major 16 x 16).
template <int RB, int CT, int SW, class S>
__device__ __forceinline__ void diag_pass(typename MT<S>::v4 (&Z)[RB][CT], const S *__restrict__ dinv,
                                          S *__restrict__ st, int wave, int nblk, int ar,
                                          int g, int i16) {
  typedef typename MT<S>::v4 v4;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int b = wave + 4 * rb;
    if (b >= nblk) continue;
    S a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = dinv[b * 256 + ar + 16 * (4 * q + g)];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) st[(4 * g + v) * SW + 16 * ct + i16] = Z[rb][ct][v];
    wave_lds_sync();
    v4 acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = MT<S>::zero();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        acc[ct] = mfma16(a[q], st[(4 * q + g) * SW + 16 * ct + i16], acc[ct]);
    wave_lds_sync();
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) Z[rb][ct] = acc[ct];
  }
}

// Z <- M^{-1} Z for one shift, Z = P^T (right-hand side) on entry: forward
// recurrence with L', diagonal pass, backward recurrence with U', diagonal pass.
// All waves of the workgroup must call it together.
template <int RB, int CT, int SW, class T_>
__device__ __forceinline__ void lu_solve_slab(typename MT<T_>::v4 (&Z)[RB][CT], const T_ *__restrict__ W,
                                              const T_ *__restrict__ dL,
                                              const T_ *__restrict__ dU, T_ (*S)[16 * SW],
                                              T_ *__restrict__ st, int np, int nblk, int wave,
                                              int ar, int g, int i16) {
    // forward recurrence with L'
#pragma unroll 1
  for (int b = 0; b < nblk; ++b) {
    T_ *Sb = S[b & 1];
    T_ a[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int bb = wave + 4 * rb;
      if (bb > b && bb < nblk) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[rb][q] = W[(16 * bb + ar) + (int64_t)(16 * b + 4 * q + g) * np];
      }
    }
    if (wave == (b & 3)) {
      const int rbo = b >> 2;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
        if (rb == rbo) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) Sb[(4 * g + v) * SW + 16 * ct + i16] = Z[rb][ct][v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int bb = wave + 4 * rb;
      if (bb > b && bb < nblk) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
            Z[rb][ct] = mfma16(-a[rb][q], Sb[(4 * q + g) * SW + 16 * ct + i16], Z[rb][ct]);
      }
    }
  }
  diag_pass<RB, CT, SW, T_>(Z, dL, st, wave, nblk, ar, g, i16);

  // backward recurrence with U'
#pragma unroll 1
  for (int b = nblk - 1; b >= 0; --b) {
    T_ *Sb = S[b & 1];
    T_ a[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int bb = wave + 4 * rb;
      if (bb < b) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[rb][q] = W[(16 * bb + ar) + (int64_t)(16 * b + 4 * q + g) * np];
      }
    }
    if (wave == (b & 3)) {
      const int rbo = b >> 2;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
        if (rb == rbo) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) Sb[(4 * g + v) * SW + 16 * ct + i16] = Z[rb][ct][v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int bb = wave + 4 * rb;
      if (bb < b) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
            Z[rb][ct] = mfma16(-a[rb][q], Sb[(4 * q + g) * SW + 16 * ct + i16], Z[rb][ct]);
      }
    }
  }
  diag_pass<RB, CT, SW, T_>(Z, dU, st, wave, nblk, ar, g, i16);

}

template <int NPMAX, int SW, bool PHI>
__global__ void __launch_bounds__(256, (NPMAX > 256 ? 1 : 2))
solve_full_f64_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist,
                      int nlist, const PlanRec *__restrict__ plan, Terms T,
                      double *__restrict__ wsd, const int *__restrict__ wsi) {
  constexpr int RB = NPMAX / 64;
  constexpr int CT = SW / 16;
  constexpr int NSLAB = NPMAX / SW;
  constexpr int PRB = PHI ? RB : 1;
  __shared__ double S[2][16 * SW];
  __shared__ double Tst[4][16 * SW];

  int slot, sl;
  xcd_map(blockIdx.x, NSLAB, slot, sl);
  if (slot >= nlist) return;
  const int ii = ilist[slot];
  if (!on_route(plan[ii], 0)) return;  // not on the pivoting LU route
  const InstDesc D = inst[ii];
  const int n = D.n, np = D.npad;
  if (np > NPMAX || (np & 15) || n > np || n < 1) return;  // sizes the host never sends
  const int c0 = sl * SW;
  const int ncol = D.ncol;
  if (c0 >= ncol) return;
  const int nblk = np >> 4;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  const double sc = ldexp(1.0, -plan[ii].s);
  const int hn = D.hn;

  v4d Z[RB][CT], Ae[RB][CT], Ap[PRB][CT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) Ae[rb][ct] = zero4();
#pragma unroll
  for (int rb = 0; rb < PRB; ++rb)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) Ap[rb][ct] = zero4();

#pragma unroll 1
  for (int k = 0; k < T.nterms; ++k) {
    const double *W = wsd + D.fac_off + (int64_t)k * np * np;
    const int *perm = wsi + D.perm_ioff + (int64_t)k * np;
    const double *dL = wsd + D.dinv_off + (int64_t)(2 * k) * nblk * 256;
    const double *dU = dL + (int64_t)nblk * 256;

    // right-hand side P^T B[:, slab], B = A 2^-s; with a folded complex weight
    // P^T emb(w B)[:, slab] = P^T (w_re B + w_im J B)[:, slab]
    const int fold = T.fold[k];
    const double fre = fold ? (T.fn[k] ? T.wp_re[k] : T.we_re[k]) : 1.0;
    const double fim = fold ? (T.fn[k] ? T.wp_im[k] : T.we_im[k]) : 0.0;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int b = wave + 4 * rb;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int col = c0 + 16 * ct + i16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * b + 4 * g + v;
          double val = 0.0;
          if (b < nblk && r < n && col < ncol) {
            const int pr = perm[r];
            if (pr < n) {
              val = D.A[(int64_t)pr * D.lda + col];
              if (fold) {
                const double aj = pr < hn ? -D.A[(int64_t)(pr + hn) * D.lda + col]
                                          : D.A[(int64_t)(pr - hn) * D.lda + col];
                val = fre * val + fim * aj;
              }
              val *= sc;
            }
          }
          Z[rb][ct][v] = val;
        }
      }
    }

    lu_solve_slab<RB, CT, SW, double>(Z, W, dL, dU, S, Tst[wave], np, nblk, wave, ar, g, i16);

    // combination in the round-off form (§4.3); folded terms already carry
    // their weight, a conjugate pair on real A adds twice the real (top) half
    const double we = fold ? 0.0 : T.we_re[k];
    const double wp = fold ? 0.0 : T.wp_re[k];
    const double fsc = T.pair_real ? 2.0 : 1.0;
    const int frows = T.pair_real ? hn : np;
    const bool fe = fold && T.fn[k] == 0, fp = fold && T.fn[k] == 1;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int r0 = 16 * (wave + 4 * rb) + 4 * g;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double z = Z[rb][ct][v];
          const double zf = (r0 + v < frows) ? fsc * z : 0.0;
          Ae[rb][ct][v] = fold ? (fe ? Ae[rb][ct][v] + zf : Ae[rb][ct][v]) : fma(we, z, Ae[rb][ct][v]);
          if constexpr (PHI) Ap[rb][ct][v] = fold ? (fp ? Ap[rb][ct][v] + zf : Ap[rb][ct][v]) : fma(wp, z, Ap[rb][ct][v]);
        }
      }
    if constexpr (PHI) {
      if (T.want_phi2) {
        // phi2 (real shift sets, never folded): sum_k wq_k Z_k accumulates in
        // its level-0 buffer, shift by shift in the order k = 0, 1, ...
        // (this workgroup's columns; no registers held across shifts)
        double *Q0 = wsd + D.r_off + 4 * (int64_t)np * np;
        const bool last = k + 1 == T.nterms;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int b = wave + 4 * rb;
          if (b >= nblk) continue;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const int col = c0 + 16 * ct + i16;
            if (col >= ncol) continue;
            const int r = 16 * b + 4 * g;
            v4d *pq = reinterpret_cast<v4d *>(Q0 + r + (int64_t)col * np);
            v4d o = k == 0 ? zero4() : *pq;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = fma(T.wq_re[k], Z[rb][ct][v], o[v]);
            if (last)
#pragma unroll
              for (int v = 0; v < 4; ++v) o[v] += (r + v == col ? T.a0q : 0.0);
            *pq = o;
          }
        }
      }
    }
    __syncthreads();
  }

  // R = a0 I + sum w_k Z_k (and Phi) into the level-0 squaring buffers
  double *R0 = wsd + D.r_off;
  double *P0 = R0 + 2 * (int64_t)np * np;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int b = wave + 4 * rb;
    if (b >= nblk) continue;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int col = c0 + 16 * ct + i16;
      if (col >= ncol) continue;
      const int r = 16 * b + 4 * g;
      v4d o = Ae[rb][ct];
#pragma unroll
      for (int v = 0; v < 4; ++v) o[v] += (r + v == col ? T.a0e : 0.0);
      *reinterpret_cast<v4d *>(R0 + r + (int64_t)col * np) = o;
      if constexpr (PHI) {
        v4d op = Ap[rb][ct];
#pragma unroll
        for (int v = 0; v < 4; ++v) op[v] += (r + v == col ? T.a0p : 0.0);
        *reinterpret_cast<v4d *>(P0 + r + (int64_t)col * np) = op;
      }
    }
  }
}

}  // namespace pfm
