// Shifted inverses X_k = (I - c_k B)^{-1} for npad = 256 by block
// Gauss-Jordan with 128-wide pivot blocks (the inverse form of §2's
// processors, combined as in §4.3 by combine_inv_kernel).
//
// Same no-interchange argument as kern_gj.h (|c_k| ||B||_1 <= 1/2 makes
// every pivot and every Schur complement column diagonally dominant), but
// two block steps instead of four: the working matrix W (column-major,
// 256 x 256 doubles) is read and written twice per inverse instead of four
// times (16 flop per byte of W traffic instead of 8, above the FP64 MFMA
// ridge).
//
// One workgroup of 8 waves per (instance, shift); wave w owns 16-row strip
// w of JJ and strip w of I.  Block step J (rows and columns JJ = [128 J, 128 J + 128),
// the rest I):
//   1. The panel W[:, JJ] is loaded into registers (two 16 x 128 strips per
//      wave, MFMA accumulator layout).
//   2. Gauss-Jordan on the panel with 16-wide pivot tiles: the pivot's owner
//      wave inverts the 16 x 16 pivot tile (one column at a time, within the
//      wave) and publishes the transformed row block in LDS; the other
//      strips take a rank-16 MFMA update from it.  The next pivot's owner
//      prepares its row block while the other waves update, so the serial
//      tile inverses overlap the products.  Afterwards JJ's strips hold
//      Dinv = W[JJ, JJ]^{-1} and I's strips hold -G = -W[I, JJ] Dinv.
//   3. Both are stored (final for these columns) and turned into MFMA A
//      fragments that stay in registers for the rest of the step.
//   4. For every 32-column chunk C outside JJ, the old row block W[JJ, C]
//      (128 x 32) is staged in LDS (double-buffered, the next chunk's loads
//      in flight during this chunk's products) and serves as the B operand
//      of both updates
//        W[JJ, C] <- Dinv W_old[JJ, C],   W[I, C] <- W_old[I, C] - G W_old[JJ, C].
// The first step reads M = I - c_k B from A directly (M is never stored).
#pragma once
#include <type_traits>
#include <utility>

#include "kern_gj.h"

namespace pfm {

constexpr int kG2 = 128;          // pivot block edge (two block steps for npad = 256)
constexpr int kG2LR = kG2 + 1;    // LDS leading dimension of a published pivot row block (16 x 128)
constexpr int kG2LS = 17;         // LDS leading dimension of a wave's 16 x 16 tile scratch
constexpr int kG2CW = 32;         // columns of a staged chunk
constexpr int kG2LC = kG2CW + 1;  // LDS leading dimension of a staged chunk
constexpr int kG2RB = 16 * kG2LR;                    // doubles per row block buffer
constexpr int kG2Panel = 3 * kG2RB + 8 * 16 * kG2LS;  // three row block buffers + 8 wave scratches
constexpr int kG2Chunks = 2 * kG2 * kG2LC;           // two staged chunks
constexpr int kG2Lds = kG2Panel > kG2Chunks ? kG2Panel : kG2Chunks;

// f(integral_constant<int, I>) for I = 0 .. N - 1, unrolled at compile time.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Workgroup barrier for LDS traffic only: this wave's LDS operations are
// complete, global stores may still be in flight (no other wave reads what
// they write before the next full __syncthreads).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Lane L of each group of 16 lanes, to every lane of that group (DPP
// row_newbcast).
template <int L>
__device__ __forceinline__ double bcast16(double d) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(d), 0x150 + L, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(d), 0x150 + L, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// 1 / d by v_rcp_f64 and two Newton steps (within an ulp or so; d is a
// pivot of a diagonally dominant matrix, far from zero and overflow).
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// One column step of a 16 x 16 Gauss-Jordan inverse without interchanges
// of a tile held by one wave in accumulator layout (element v of lane
// (g, i) = T[4 g + v][i]), in registers: pivot column C from lane C of each
// 16-lane group (DPP), pivot row C from group C / 4 (lane shuffle).
template <int C>
__device__ __forceinline__ void gj16_col(v4d &x, int g, int i16) {
  double pcol[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) pcol[v] = bcast16<C>(x[v]);  // T[4 g + v][C]
  const double pr = __shfl(x[C & 3], 16 * (C >> 2) + i16);  // T[C][i]
  const double piv = bcast16<C>(pr);                        // T[C][C]
  const double pinv = recip(piv);
  const double rp = pr * pinv;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * g + v;
    double nv = fma(-pcol[v], rp, x[v]);
    nv = i16 == C ? -pcol[v] * pinv : nv;
    nv = r == C ? rp : nv;
    nv = (r == C && i16 == C) ? pinv : nv;
    x[v] = nv;
  }
}

// ACT: B = A / N (the action's steps) instead of A 2^-s.  Instances with
// npad != 256 are left to gj_inv_kernel.
template <bool ACT>
__global__ void __launch_bounds__(512)
gj2_inv_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nlist,
               PlanRec *__restrict__ plan, Terms T, double *__restrict__ wsd, int route_val) {
  constexpr int NP = 256, LR = kG2LR, LS = kG2LS, LC = kG2LC;
  __shared__ double lds[kG2Lds];
  int slot, k;
  xcd_map(blockIdx.x, T.nterms, slot, k);
  if (slot >= nlist) return;
  const int ii = ilist[slot];
  if (!on_route(plan[ii], route_val)) return;  // uniform per workgroup
  const InstDesc D = inst[ii];
  if (D.npad != NP || D.n > NP || D.n < 1) return;
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  double *W = wsd + D.fac_off + (int64_t)k * NP * NP;
  const ShiftedA<ACT> M0{D.A, D.lda, D.n, T.c_re[k], ldexp(T.c_re[k], -plan[ii].s), (double)plan[ii].s};
  double *Ss = lds + 3 * kG2RB + w * 16 * LS;  // this wave's tile scratch
  double *Cl0 = lds, *Cl1 = lds + kG2 * LC;

  // A fragments of a 16 x 16 tile held in accumulator layout (element v of
  // lane (g, i) = tile[4 g + v][i]): element kk of lane (g, i) becomes
  // tile[ar(i)][4 kk + g], the operand of k-step kk (k = 4 kk + g).
  auto to_afrag = [&](const v4d &c) -> v4d {
#pragma unroll
    for (int v = 0; v < 4; ++v) Ss[(4 * g + v) * LS + i16] = c[v];
    wave_lds_sync();
    v4d a;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) a[kk] = Ss[ar * LS + 4 * kk + g];
    wave_lds_sync();
    return a;
  };

  auto step = [&](auto first_tag) {
    constexpr bool FIRST = decltype(first_tag)::value;
    constexpr int j0 = FIRST ? 0 : kG2;  // JJ
    constexpr int o0 = FIRST ? kG2 : 0;  // I (rows), and the columns outside JJ
    const int rj = j0 + 16 * w, ri = o0 + 16 * w;  // this wave's strips

    // 1. this wave's strips of the panel W[:, JJ]: 8 tiles of 16 x 16 each,
    //    accumulator layout (element v of lane (g, i): row r + 4 g + v,
    //    column j0 + 16 q + i)
    v4d SJ[8], SI[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if constexpr (FIRST) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          SJ[q][v] = M0(rj + 4 * g + v, j0 + 16 * q + i16);
          SI[q][v] = M0(ri + 4 * g + v, j0 + 16 * q + i16);
        }
      } else {
        SJ[q] = *reinterpret_cast<const v4d *>(W + (rj + 4 * g) + (j0 + 16 * q + i16) * NP);
        SI[q] = *reinterpret_cast<const v4d *>(W + (ri + 4 * g) + (j0 + 16 * q + i16) * NP);
      }
    }

    // 2. Gauss-Jordan on the panel with 16-wide pivot tiles.  Pivot p lives
    //    in wave p's JJ strip; its owner inverts the pivot tile and
    //    publishes the transformed row block R_p (tile p = the inverse) in
    //    buffer p & 1; every other strip then does
    //      S[:, q] -= S[:, p] R_p[:, q]  (q != p),   S[:, p] <- -S[:, p] R_p[:, p].
    //    The owner of p + 1 updates its JJ strip first and then, at raised
    //    priority, inverts tile p + 1 and publishes R_{p+1} while the other
    //    waves update: the serial tile inverses overlap the products.  One barrier per pivot;
    //    R_{p+1} goes to the buffer last read before the previous barrier.

    // The owner of pivot P publishes, in buffer P & 1, its JJ strip (the
    // row block of pivot P, updated with the earlier pivots) with tile P
    // replaced by x = Tinv, its inverse.  Only LDS is written.
    auto publish = [&](auto Pc, const v4d &x) {
      constexpr int P = decltype(Pc)::value;
      double *Rb = lds + (P % 3) * kG2RB;
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) Rb[(4 * g + v) * LR + 16 * q + i16] = q == P ? x[v] : SJ[q][v];
    };
    // Pivot p (Tinv = the inverse of pivot tile p, Row = its row block, both
    // from buffer p & 1).  A strip S other than the row block itself:
    //   G = S[:, p] Tinv,  S[:, q] -= G Row[:, q] (q != p),  S[:, p] = -G;
    // the row block's own strip (keep): S[:, q] = Tinv Row[:, q], S[:, p] = Tinv.
    // All waves run the same program: tile p + 1 of the JJ strip first, so
    // that the owner of p + 1 can invert it (VALU work in a branch that
    // touches only its copy x) while the MFMA pipe serves the other waves;
    // then the rest of both strips.  No strip register is written on one
    // side of a branch only.
    auto pivot = [&](auto pc) {
      constexpr int p = decltype(pc)::value;
      constexpr int P = p + 1;
      const double *R = lds + (p % 3) * kG2RB;
      const bool keep = w == p;
      const bool next = P < 8 && w == P;
      // multipliers M (A fragments) of a strip for the pivot published in
      // Rp (tile pp = Tinv), and its new tile pp
      auto strip_mult = [&](v4d(&S)[8], const double *Rp, auto ppc, bool kp) -> v4d {
        constexpr int pp = decltype(ppc)::value;
        v4d tf, tc;  // Tinv as A fragments and in accumulator layout
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) tf[kk] = Rp[ar * LR + 16 * pp + 4 * kk + g];
#pragma unroll
        for (int v = 0; v < 4; ++v) tc[v] = Rp[(4 * g + v) * LR + 16 * pp + i16];
        const v4d a = to_afrag(S[pp]);
        v4d G = zero4();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) G = mfma16(a[kk], Rp[(4 * kk + g) * LR + 16 * pp + i16], G);
        const v4d gf = to_afrag(G);
        v4d M;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) M[kk] = kp ? tf[kk] : -gf[kk];
#pragma unroll
        for (int v = 0; v < 4; ++v) S[pp][v] = kp ? tc[v] : -G[v];
        return M;
      };
      auto tile = [&](v4d(&S)[8], const double *Rp, const v4d &M, bool kp, auto qc) {
        constexpr int q = decltype(qc)::value;
        v4d acc = S[q];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = kp ? 0.0 : acc[v];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = mfma16(M[kk], Rp[(4 * kk + g) * LR + 16 * q + i16], acc);
        S[q] = acc;
      };
      // the whole I strip for pivot pp
      auto si_update = [&](const double *Rp, auto ppc) {
        constexpr int pp = decltype(ppc)::value;
        const v4d MI = strip_mult(SI, Rp, ppc, false);
        static_for<8>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          if constexpr (q != pp) tile(SI, Rp, MI, false, qc);
          if constexpr (q & 1) __builtin_amdgcn_sched_barrier(0);
        });
      };
      // the owner of p deferred its I strip's update for pivot p - 1
      if constexpr (p > 0) {
        if (keep) si_update(lds + ((p - 1) % 3) * kG2RB, std::integral_constant<int, p - 1>{});
      }
      if (next) __builtin_amdgcn_s_setprio(2);
      const v4d MJ = strip_mult(SJ, R, pc, keep);
      if constexpr (P < 8) {
        tile(SJ, R, MJ, keep, std::integral_constant<int, P>{});
        v4d x = SJ[P];
        if (next) static_for<16>([&](auto cc) { gj16_col<decltype(cc)::value>(x, g, i16); });
        static_for<8>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          if constexpr (q != p && q != P) tile(SJ, R, MJ, keep, qc);
          if constexpr (q & 1) __builtin_amdgcn_sched_barrier(0);
        });
        if (next) publish(std::integral_constant<int, P>{}, x);
        if (next) __builtin_amdgcn_s_setprio(0);
        // the next pivot's owner defers its I strip's update to pivot p + 1
        if (!next) si_update(R, pc);
      } else {
        static_for<8>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          if constexpr (q != p) tile(SJ, R, MJ, keep, qc);
          if constexpr (q & 1) __builtin_amdgcn_sched_barrier(0);
        });
        si_update(R, pc);
      }
      lds_barrier();
    };
    if (w == 0) {
      v4d x = SJ[0];
      static_for<16>([&](auto cc) { gj16_col<decltype(cc)::value>(x, g, i16); });
      publish(std::integral_constant<int, 0>{}, x);
    }
    lds_barrier();
    pivot(std::integral_constant<int, 0>{});
    pivot(std::integral_constant<int, 1>{});
    pivot(std::integral_constant<int, 2>{});
    pivot(std::integral_constant<int, 3>{});
    pivot(std::integral_constant<int, 4>{});
    pivot(std::integral_constant<int, 5>{});
    pivot(std::integral_constant<int, 6>{});
    pivot(std::integral_constant<int, 7>{});

    // 3. the strips are final for the columns JJ (Dinv rows, -G): store
    //    them, then keep them as A fragments, M[tt][kk] = strip[ar(i)][16 tt + 4 kk + g]
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      *reinterpret_cast<v4d *>(W + (rj + 4 * g) + (j0 + 16 * q + i16) * NP) = SJ[q];
      *reinterpret_cast<v4d *>(W + (ri + 4 * g) + (j0 + 16 * q + i16) * NP) = SI[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      SJ[q] = to_afrag(SJ[q]);
      SI[q] = to_afrag(SI[q]);
    }
    lds_barrier();  // the panel buffers become the two chunk buffers

    // 4. chunks of 32 columns outside JJ:
    //    W[JJ, C] <- Dinv W_old[JJ, C],  W[I, C] <- W_old[I, C] + (-G) W_old[JJ, C]
    double stg[8];
    auto load_stage = [&](int ch) {
      const int cbase = o0 + kG2CW * ch;
      if constexpr (FIRST) {  // row-major A: coalesced along the columns
        const int c = t & 31, rr = t >> 5;
#pragma unroll
        for (int u = 0; u < 8; ++u) stg[u] = M0(j0 + rr + 16 * u, cbase + c);
      } else {
        const int r = t & 127, c0 = t >> 7;
#pragma unroll
        for (int u = 0; u < 8; ++u) stg[u] = W[(j0 + r) + (cbase + c0 + 4 * u) * NP];
      }
    };
    auto stage = [&](double *Cl) {
      if constexpr (FIRST) {
        const int c = t & 31, rr = t >> 5;
#pragma unroll
        for (int u = 0; u < 8; ++u) Cl[(rr + 16 * u) * LC + c] = stg[u];
      } else {
        const int r = t & 127, c0 = t >> 7;
#pragma unroll
        for (int u = 0; u < 8; ++u) Cl[r * LC + c0 + 4 * u] = stg[u];
      }
    };
    // the I strip's old values of a chunk, W_old[I, C]
    v4d nxt[2];
    auto load_old = [&](int ch) {
      const int cbase = o0 + kG2CW * ch;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if constexpr (FIRST) {
#pragma unroll
          for (int v = 0; v < 4; ++v) nxt[b][v] = M0(ri + 4 * g + v, cbase + 16 * b + i16);
        } else {
          nxt[b] = *reinterpret_cast<const v4d *>(W + (ri + 4 * g) + (cbase + 16 * b + i16) * NP);
        }
      }
    };
    load_stage(0);
    load_old(0);
    stage(Cl0);
    lds_barrier();
    constexpr int NCH = (NP - kG2) / kG2CW;
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
      const double *Cl = (ch & 1) ? Cl1 : Cl0;
      const int cbase = o0 + kG2CW * ch;
      v4d aj[2] = {zero4(), zero4()}, ai[2] = {nxt[0], nxt[1]};
      if (ch + 1 < NCH) {  // in flight during the products
        load_stage(ch + 1);
        load_old(ch + 1);
      }
#pragma unroll
      for (int tt = 0; tt < 8; ++tt)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const double bv = Cl[(16 * tt + 4 * kk + g) * LC + 16 * b + i16];
            aj[b] = mfma16(SJ[tt][kk], bv, aj[b]);
            ai[b] = mfma16(SI[tt][kk], bv, ai[b]);
          }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        *reinterpret_cast<v4d *>(W + (rj + 4 * g) + (cbase + 16 * b + i16) * NP) = aj[b];
        *reinterpret_cast<v4d *>(W + (ri + 4 * g) + (cbase + 16 * b + i16) * NP) = ai[b];
      }
      if (ch + 1 < NCH) stage((ch & 1) ? Cl0 : Cl1);
      lds_barrier();
    }
  };
  step(std::true_type{});
  __syncthreads();  // step 0's stores are read by other waves in step 1
  step(std::false_type{});
}

}  // namespace pfm
