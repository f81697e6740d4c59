// Shifted inverses X_k = (I - c_k B)^{-1} by block Gauss-Jordan, for
// instances where partial pivoting provably performs no interchange.
//
// With |c_k| ||B||_1 < 1, M_k = I - c_k B is strictly column diagonally
// dominant (|1 - c_k b_jj| >= 1 - |c_k| |b_jj| > |c_k| sum_{i != j} |b_ij|), and
// elimination keeps it so: every multiplier has |l_ij| < 1 and the partial
// pivoting choice (largest |.| in the column, first index on ties) is always
// the diagonal.  The host sends an instance here only if |c_k| ||B||_1 <= 1/2
// for every shift (the planner's ||B||_1 <= θ gives |c_k| ||B||_1 < 0.06 on
// the paper's sets); anything else takes the pivoting LU path.  The inverse
// then serves §2's "inverse" form of each processor, (I - c_k B)^{-1}, and the
// round-off combination of §4.3 becomes
//   R = a0 I + (sum_k w_k X_k) B,
// one product per instance instead of one solve per shift.
//
// Algorithm (in place, column-major, npad a multiple of 64, blocks of 64):
//   for each block J:  D = W[J,J];  Dinv = D^{-1} (Gauss-Jordan in LDS)
//     W[J,c] <- Dinv W[J,c]            (c != J)   MFMA, Dinv from LDS
//     W[I,c] <- W[I,c] - W[I,J] W[J,c] (I,c != J) MFMA rank-64 update
//     W[I,J] <- -W[I,J] Dinv           (I != J)
//     W[J,J] <- Dinv
// Each wave keeps its 16-row strips of W[I,J] in registers (MFMA A operand)
// for the whole step; each 64-column chunk of the transformed row block is
// staged once in LDS and is the B operand of the update, so the inner loops
// read only registers and LDS.  M itself is never stored: the first step
// reads its elements from A as it goes (the update is bound by memory
// traffic, and this saves one write and one read of the whole matrix).
#pragma once
#include <type_traits>

#include "kern_common.h"

namespace pfm {

constexpr int kGJ = 64;

// Element (r, c) of M = I - c_k B (B = A 2^-s, or A / N for the action) of
// a real non-embedded instance, from row-major A; identity in the padding.
template <bool ACT>
struct ShiftedA {
  const double *A;
  int64_t lda;
  int n;
  double ck, cs, Nd;
  __device__ __forceinline__ double operator()(int r, int c) const {
    const double a = (r < n && c < n) ? A[(int64_t)r * lda + c] : 0.0;
    const double cb = ACT ? ck * (a / Nd) : cs * a;
    return (r == c ? 1.0 : 0.0) - cb;
  }
};

// 64 x 64 Gauss-Jordan inverse without interchanges of the block held
// row-major in LDS (leading dimension LDD), in place.  Each of the 256
// threads keeps its 4 x 4 patch (rows pr0.., columns pc0..) in registers for
// all 64 columns; the current pivot column and row are broadcast through the
// double-buffered bcc / bcr arrays (2 x 64 each), one barrier per column.
// The caller synchronises before reading Dl afterwards.
template <int LDD>
__device__ __forceinline__ void gj64_regs(double *Dl, double *bcc, double *bcr, int pr0, int pc0) {
  double x[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) x[a][b] = Dl[(pr0 + a) * LDD + pc0 + b];
  if (pc0 == 0)
#pragma unroll
    for (int a = 0; a < 4; ++a) bcc[pr0 + a] = x[a][0];
  if (pr0 == 0)
#pragma unroll
    for (int b = 0; b < 4; ++b) bcr[pc0 + b] = x[0][b];
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < 64; ++c) {
    const double *cc = bcc + (c & 1) * 64, *cr = bcr + (c & 1) * 64;
    const double p = 1.0 / cc[c];
    double colc[4], rp[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) colc[a] = cc[pr0 + a];
#pragma unroll
    for (int b = 0; b < 4; ++b) rp[b] = cr[pc0 + b] * p;  // the pivot row scaled
    // every element as if outside the pivot row and column ...
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) x[a][b] = fma(-colc[a], rp[b], x[a][b]);
    // ... then the pivot row (scaled), column (-colc p) and element (p)
    // rewritten by their owners; c & 3 is the same in every lane
    const bool own_r = pr0 == (c & ~3), own_c = pc0 == (c & ~3);
#define PFM_GJ_FIX(Q)                                                         \
  {                                                                           \
    if (own_r)                                                                \
      for (int b = 0; b < 4; ++b) x[Q][b] = rp[b];                            \
    if (own_c)                                                                \
      for (int a = 0; a < 4; ++a) x[a][Q] = -colc[a] * p;                     \
    if (own_r && own_c) x[Q][Q] = p;                                          \
  }
    switch (c & 3) {
      case 0: PFM_GJ_FIX(0) break;
      case 1: PFM_GJ_FIX(1) break;
      case 2: PFM_GJ_FIX(2) break;
      default: PFM_GJ_FIX(3) break;
    }
#undef PFM_GJ_FIX
    const int cn = c + 1;  // owners of column / row c + 1 broadcast it
    if (cn < 64) {
      double *nc = bcc + (cn & 1) * 64, *nr = bcr + (cn & 1) * 64;
      const bool on_c = (cn >> 2) == (pc0 >> 2), on_r = (cn >> 2) == (pr0 >> 2);
#define PFM_GJ_BC(Q)                                                          \
  {                                                                           \
    if (on_c)                                                                 \
      for (int a = 0; a < 4; ++a) nc[pr0 + a] = x[a][Q];                      \
    if (on_r)                                                                 \
      for (int b = 0; b < 4; ++b) nr[pc0 + b] = x[Q][b];                      \
  }
      switch (cn & 3) {
        case 0: PFM_GJ_BC(0) break;
        case 1: PFM_GJ_BC(1) break;
        case 2: PFM_GJ_BC(2) break;
        default: PFM_GJ_BC(3) break;
      }
#undef PFM_GJ_BC
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Dl[(pr0 + a) * LDD + pc0 + b] = x[a][b];
}

// ACT: B = A / N (the action's steps) instead of A 2^-s.
template <int NPMAX, bool ACT>
__global__ void __launch_bounds__(256, 2)
gj_inv_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nlist,
              PlanRec *__restrict__ plan, Terms T, double *__restrict__ wsd, int route_val) {
  constexpr int LDD = kGJ + 1;
  __shared__ double Dl[kGJ * LDD];      // D, then D^{-1} (row-major, padded)
  __shared__ double Cl[kGJ * LDD];      // staging for the row-block product
  __shared__ double bcc[2 * kGJ], bcr[2 * kGJ];  // pivot column / row broadcast

  int slot, k;
  xcd_map(blockIdx.x, T.nterms, slot, k);
  if (slot >= nlist) return;
  const int ii = ilist[slot];
  if (!on_route(plan[ii], route_val)) return;  // the device chose another route (uniform per workgroup)
  const InstDesc D = inst[ii];
  const int np = D.npad;
  if (np > NPMAX || (np % kGJ) || D.n > np || D.n < 1) return;  // never sent
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  double *W = wsd + D.fac_off + (int64_t)k * np * np;  // 32-bit offsets below: npad <= 512
  const int nJ = np / kGJ;

  const ShiftedA<ACT> M0{D.A, D.lda, D.n, T.c_re[k], ldexp(T.c_re[k], -plan[ii].s), (double)plan[ii].s};

  // this thread's 4 x 4 patch of a 64 x 64 block, and its place in
  // coalesced block copies (one row per lane, columns (t >> 6) + 4 u)
  const int pr0 = (t >> 4) * 4, pc0 = (t & 15) * 4;
  const int cr = t & 63, cc0 = t >> 6;

  // one block step; the first reads M from A (FIRST), the others from W
  auto step = [&](const int J, auto first_tag) {
    constexpr bool FIRST = decltype(first_tag)::value;
    const int j0 = J * kGJ;
    // 1. Dinv in LDS by Gauss-Jordan without interchanges
    if constexpr (FIRST) {
#pragma unroll
      for (int u = 0; u < 16; ++u) Dl[(cc0 + 4 * u) * LDD + cr] = M0(cc0 + 4 * u, cr);
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u)
        Dl[cr * LDD + cc0 + 4 * u] = W[(j0 + cr) + (j0 + cc0 + 4 * u) * np];
    }
    __syncthreads();
    gj64_regs<LDD>(Dl, bcc, bcr, pr0, pc0);
    __syncthreads();

    // Strips of 16 rows outside block J, strip w + 4 m to wave w, MSG per
    // wave at a time (NG groups).  With G = W[I, J] Dinv, the step is
    //   W[I, C] <- W[I, C] - G W_old[J, C]   (C != J)
    //   W[J, C] <- Dinv W_old[J, C]          (C != J)
    //   W[I, J] <- -G,  W[J, J] <- Dinv,
    // so the transform of the row block and the update of the other rows
    // read the same staged old chunk and are independent of each other.
    // G comes out of G^T = Dinv^T W[I, J]^T, whose accumulator layout is
    // the MFMA A-fragment layout the update needs: lane (g, i) holds
    // G[row ar(i)][16 t + 4 g + v] in element v of tile t, which is the A
    // operand of k-step q = 4 t + v when the B operand supplies chunk row
    // 16 t + 4 g + v.  With several groups, only the last transforms the row
    // block, so earlier groups still see the old chunk.
    constexpr int MSW = NPMAX / 64 - 1 > 0 ? NPMAX / 64 - 1 : 1;  // strips per wave, at most
    constexpr int MSG = MSW < 3 ? MSW : (NPMAX >= 512 ? 2 : 3);    // register budget
    constexpr int NG = (MSW + MSG - 1) / MSG;
    const int nstrip = (np - kGJ) / 16;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
    const int wu = __builtin_amdgcn_readfirstlane(wave);
#pragma unroll 1
    for (int grp = 0; grp < NG; ++grp) {
      v4d Gt[MSG][4];  // G of each strip, 4 tiles of 16 columns
      int srow[MSG];
#pragma unroll
      for (int m = 0; m < MSG; ++m) {
        const int sidx = wu + 4 * (grp * MSG + m);
        srow[m] = sidx < nstrip ? sidx * 16 + (sidx * 16 >= j0 ? kGJ : 0) : -1;
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) Gt[m][tt] = zero4();
        if (srow[m] < 0) continue;
        const int r0 = srow[m];
        // G^T tile tt = (Dinv^T)[16 tt.., :] W[I, J]^T : A = Dinv^T rows
        // 16 tt + ar(i) (= Dinv columns), B = W[r0 + ar(j), j0 + k]
#pragma unroll
        for (int q = 0; q < kGJ / 4; ++q) {
          const double bv = FIRST ? M0(r0 + ar, 4 * q + g) : W[(r0 + ar) + (j0 + 4 * q + g) * np];
#pragma unroll
          for (int tt = 0; tt < 4; ++tt)
            Gt[m][tt] = mfma16(Dl[(4 * q + g) * LDD + 16 * tt + ar], bv, Gt[m][tt]);
        }
        // new W[I, J] = -G: lane (g, i) holds row r0 + ar(i), columns 16 tt + 4 g + v
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
          for (int v = 0; v < 4; ++v) W[(r0 + ar) + (j0 + 16 * tt + 4 * g + v) * np] = -Gt[m][tt][v];
      }

#pragma unroll 1
      for (int C = 0; C < nJ; ++C) {
        if (C == J) continue;
        const int c0 = C * kGJ;
        if constexpr (FIRST) {
#pragma unroll
          for (int u = 0; u < 16; ++u) Cl[(cc0 + 4 * u) * LDD + cr] = M0(cc0 + 4 * u, c0 + cr);
        } else {
#pragma unroll
          for (int u = 0; u < 16; ++u)
            Cl[cr * LDD + cc0 + 4 * u] = W[(j0 + cr) + (c0 + cc0 + 4 * u) * np];
        }
        __syncthreads();
        if (grp == NG - 1) {
          // W[J, C] <- Dinv W_old[J, C]: this wave's 32 x 32 part
          v4d acc[2][2];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = zero4();
#pragma unroll 4
          for (int q = 0; q < kGJ / 4; ++q) {
            const int kk = 4 * q + g;
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = Dl[(wr + 16 * a + ar) * LDD + kk];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Cl[kk * LDD + wc + 16 * b + i16];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
              for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
          }
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              *reinterpret_cast<v4d *>(W + (j0 + wr + 16 * a + 4 * g) + (c0 + wc + 16 * b + i16) * np) = acc[a][b];
        }
        // W[I, C] -= G W_old[J, C] for this wave's strips
#pragma unroll
        for (int m = 0; m < MSG; ++m) {
          if (srow[m] < 0) continue;
          const int r0 = srow[m];
          v4d cacc[4];
          if constexpr (FIRST) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
              for (int v = 0; v < 4; ++v) cacc[b][v] = M0(r0 + 4 * g + v, c0 + 16 * b + i16);
          } else {
#pragma unroll
            for (int b = 0; b < 4; ++b)
              cacc[b] = *reinterpret_cast<const v4d *>(W + (r0 + 4 * g) + (c0 + 16 * b + i16) * np);
          }
#pragma unroll
          for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
              for (int b = 0; b < 4; ++b)
                cacc[b] = mfma16(-Gt[m][tt][v], Cl[(16 * tt + 4 * g + v) * LDD + 16 * b + i16], cacc[b]);
#pragma unroll
          for (int b = 0; b < 4; ++b)
            *reinterpret_cast<v4d *>(W + (r0 + 4 * g) + (c0 + 16 * b + i16) * np) = cacc[b];
        }
        __syncthreads();  // before the next chunk overwrites Cl
      }
    }
    // 5. W[J, J] <- Dinv
#pragma unroll
    for (int u = 0; u < 16; ++u)
      W[(j0 + cr) + (j0 + cc0 + 4 * u) * np] = Dl[cr * LDD + cc0 + 4 * u];
    __syncthreads();
  };
  step(0, std::true_type{});
#pragma unroll 1
  for (int J = 1; J < nJ; ++J) step(J, std::false_type{});
}

// S_e = sum_k we_k X_k, S_p = sum_k wp_k X_k (and S_q = sum_k wq_k X_k for
// phi2) (binary64, fixed order k = 0..),
// into the level-1 squaring buffers (free at this point).  Large instances
// (route 2) take the weights w_k c_k instead: T = sum_k w_k c_k X_k for the
// form R = a0 I + alpha1 B + B T B (see square_level_f64_kernel).  The
// hybrid set of §4.3 adds d1 B + d2 B^2 to R: here S_e + d1 I + d2 B (so that
// the product gives it), or T + d2 I on route 2 (its d1 joins alpha1).  Grid:
// x = chunk of 4 * 256 elements, y = instance.
__global__ void __launch_bounds__(256)
combine_inv_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, Terms T,
                   double *__restrict__ wsd, const PlanRec *__restrict__ plan) {
  const int ii = ilist[blockIdx.y];
  if (!on_route(plan[ii], 1) && !on_route(plan[ii], 2)) return;
  const InstDesc D = inst[ii];
  const int64_t nn = (int64_t)D.npad * D.npad;
  const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (e0 >= nn) return;
  const double *X = wsd + D.fac_off;
  const bool q1 = plan[ii].route == 2;
  v4d se = zero4(), sp = zero4(), sq = zero4();
  for (int k = 0; k < T.nterms; ++k) {
    const v4d x = *reinterpret_cast<const v4d *>(X + (int64_t)k * nn + e0);
    const double we = q1 ? T.we_re[k] * T.c_re[k] : T.we_re[k];
    const double wp = q1 ? T.wp_re[k] * T.c_re[k] : T.wp_re[k];
    const double wq = T.wq_re[k];  // phi2: real full instances on route 1 only
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      se[v] = fma(we, x[v], se[v]);
      sp[v] = fma(wp, x[v], sp[v]);
      sq[v] = fma(wq, x[v], sq[v]);
    }
  }
  if (T.d1e != 0.0 || T.d2e != 0.0) {
    const int s = plan[ii].s, np = D.npad;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t e = e0 + v;
      const int r = (int)(e % np), c = (int)(e / np);
      if (q1) {
        if (r == c) se[v] += T.d2e;
      } else {
        const double b = (r < D.n && c < D.n) ? ldexp(D.A[(int64_t)r * D.lda + c], -s) : 0.0;
        se[v] += (r == c ? T.d1e : 0.0) + T.d2e * b;
      }
    }
  }
  double *base = wsd + D.r_off;
  *reinterpret_cast<v4d *>(base + nn + e0) = se;                    // R buffer 1
  if (T.want_phi) *reinterpret_cast<v4d *>(base + 3 * nn + e0) = sp;  // Phi buffer 1
  if (T.want_phi2) *reinterpret_cast<v4d *>(base + 5 * nn + e0) = sq; // Phi2 buffer 1
}

}  // namespace pfm
