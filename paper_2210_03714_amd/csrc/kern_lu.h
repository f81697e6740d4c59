// Batched LU with partial pivoting of the shifted matrices M_k = I - c_k B.
//
// §2: each "processor" k needs (I - c_k B)^{-1} applied to a right-hand side;
// a dense shifted inverse costs an LU decomposition plus triangular solves
// (§1, first item of the cost list).  One workgroup factors one (instance,
// shift) pair; the shift is applied while the matrix is loaded, so M_k is
// never formed in memory separately.
//
// Storage: the factors of M_k (not of its transpose) in column-major order
// with leading dimension npad (n rounded up to a multiple of 16, padded with
// the identity so that no kernel needs a ragged tail).  L is unit lower, U
// upper; the row interchanges are applied to the whole rows (LAPACK getrf
// convention) and summarised as a permutation perm: (P^T M)[r] = M[perm[r]].
// The 16x16 diagonal blocks of L and U are also stored inverted, for the
// MFMA block solves of the solve kernels.
//
// Algorithm: right-looking blocked LU with panel width 16.
//   panel     rows j0.., 16 columns, one row per thread in registers; pivot =
//             first index of max |x| (LAPACK idamax rule): a shuffle
//             reduction per wave, then each wave posts its candidate row to a
//             double-buffered LDS slot, so one barrier per column suffices;
//   swaps     applied to all columns outside the panel;
//   U12       = L11^{-1} A12, one column per thread;
//   A22      -= L21 U12 on v_mfma_f64_16x16x4 with L21, U12 from LDS, eight
//             16x16 tiles in flight per wave.
// Epilogue for the solve kernels: the 16x16 diagonal blocks of L and U are
// inverted (stored separately) and every off-diagonal block is multiplied by
// the inverse of the diagonal block of its column:
//   L'_ij = L_ij inv(L_jj) (i > j),   U'_ij = U_ij inv(U_jj) (i < j).
// A block substitution then runs on un-normalised blocks (the diagonal solves
// leave the critical path; see the solve kernel).
#pragma once
#include "kern_common.h"

namespace pfm {

template <int NPMAX, class S>
__global__ void __launch_bounds__(256, (NPMAX > 256 ? 1 : 2))
lu_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist,
              int nlist, PlanRec *__restrict__ plan, Terms T,
              double *__restrict__ wsd, int *__restrict__ wsi, int action) {
  constexpr int H = (NPMAX + 255) / 256;
  constexpr int LDP = NPMAX + 16;  // panel column stride in LDS (== 16 mod 32)
  constexpr int LDU = NPMAX + 16;  // U12 row stride in LDS
  constexpr int NOIDX = 0x7fffffff;
  typedef typename MT<S>::v4 v4;
  // panel and U12 share one LDS block with the load phase's two 32x33
  // binary64 staging tiles (2 x 1056 doubles, smaller than panel + U12)
  constexpr int kPanelBytes = 16 * LDP * (int)sizeof(S);
  constexpr int kSmemBytes = 2 * kPanelBytes;
  static_assert(kSmemBytes >= 2 * 1056 * 8, "staging tiles must fit");
  __shared__ __align__(16) char smem[kSmemBytes];
  S *panel = reinterpret_cast<S *>(smem);
  S *u12 = reinterpret_cast<S *>(smem + kPanelBytes);
  __shared__ S cand[2][4][18];  // per column parity and wave: row, |pivot|, index
  __shared__ S qbuf[2][16];
  __shared__ int ipiv_s[16];
  __shared__ int anyswap_s;

  int slot, k;
  xcd_map(blockIdx.x, T.nterms, slot, k);
  if (slot >= nlist) return;
  const int ii = ilist[slot];
  if (!on_route(plan[ii], 0)) return;  // the device chose another route (uniform per workgroup)
  const InstDesc D = inst[ii];
  const int n = D.n, np = D.npad;
  if (np > NPMAX || (np & 15) || n > np || n < 1) return;  // sizes the host never sends
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = MT<S>::arow_(i16);

  S *W = reinterpret_cast<S *>(wsd + D.fac_off) + (int64_t)k * np * np;
  int *ipiv = wsi + D.ipiv_ioff + (int64_t)k * np;
  int *perm = wsi + D.perm_ioff + (int64_t)k * np;
  const int nblk = np >> 4;
  S *dL = reinterpret_cast<S *>(wsd + D.dinv_off) + (int64_t)(2 * k) * nblk * 256;
  S *dU = dL + (int64_t)nblk * 256;

  const PlanRec P = plan[ii];
  const double c = T.c_re[k];
  const double cs = ldexp(c, -P.s);          // full matrix: c 2^-s (exact)
  const double Nd = (double)P.s;              // action: P.s holds N

  if (t == 0) anyswap_s = 0;

  // 1. W = I - c B, B = A 2^-s (or A / N), transposed from row-major A.  For
  //    a complex shift on an embedded instance, c B = c_re B + c_im J B with
  //    (J B)[r] = -B[r + hn] (r < hn), B[r - hn] (r >= hn).
  {
    const double ci = T.c_im[k];
    const bool jterm = D.emb && ci != 0.0;
    const double csi = ldexp(ci, -P.s);
    double *tile = reinterpret_cast<double *>(smem);   // 32 x 33 staging tile
    double *tilej = tile + 1056;                        // J B staging tile
    for (int tr = 0; tr < np; tr += 32) {
      for (int tc = 0; tc < np; tc += 32) {
        const int rl = t >> 3, cl = (t & 7) * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = tr + rl, cc = tc + cl + u;
          const bool ok = r < n && cc < n;
          tile[rl * 33 + cl + u] = ok ? D.A[(int64_t)r * D.lda + cc] : 0.0;
          if (jterm) {
            const int hn = D.hn;
            tilej[rl * 33 + cl + u] =
                ok ? (r < hn ? -D.A[(int64_t)(r + hn) * D.lda + cc] : D.A[(int64_t)(r - hn) * D.lda + cc])
                   : 0.0;
          }
        }
        __syncthreads();
        const int cc = tc + rl;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = tr + cl + u;
          if (r < np && cc < np) {
            const double a = tile[(cl + u) * 33 + rl];
            double cb = action ? c * (a / Nd) : cs * a;
            if (jterm) {
              const double aj = tilej[(cl + u) * 33 + rl];
              cb += action ? ci * (aj / Nd) : csi * aj;
            }
            W[r + (int64_t)cc * np] = (S)((r == cc ? 1.0 : 0.0) - cb);
          }
        }
        __syncthreads();
      }
    }
  }

  // 2. Blocked right-looking factorisation.
  for (int j0 = 0; j0 < np; j0 += 16) {
    S pr[H][16];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int r = j0 + t + 256 * h;
#pragma unroll
      for (int cc = 0; cc < 16; ++cc)
        pr[h][cc] = (r < np) ? W[r + (int64_t)(j0 + cc) * np] : 0.0;
    }
#pragma unroll
    for (int c2 = 0; c2 < 16; ++c2) {
      const int qrow = j0 + c2;
      const int par = c2 & 1;
      S best = -1;
      int bi = NOIDX;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int r = j0 + t + 256 * h;
        if (r >= qrow && r < np) {
          const S a = fabs(pr[h][c2]);
          if (a > best) { best = a; bi = r; }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const S ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      // the lane holding this wave's candidate posts it (row values included)
      if (bi == NOIDX) {
        if (lane == 0) { cand[par][wave][16] = -1; cand[par][wave][17] = (S)-1; }
      } else {
#pragma unroll
        for (int h = 0; h < H; ++h) {
          if (j0 + t + 256 * h == bi) {
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) cand[par][wave][cc] = pr[h][cc];
            cand[par][wave][16] = best;
            cand[par][wave][17] = (S)bi;
          }
        }
      }
      if (t == c2) {
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) qbuf[par][cc] = pr[0][cc];
      }
      __syncthreads();
      best = cand[par][0][16];
      bi = cand[par][0][17] < 0 ? NOIDX : (int)cand[par][0][17];
      int wsel = 0;
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        const S ob = cand[par][w][16];
        const int oi = cand[par][w][17] < 0 ? NOIDX : (int)cand[par][w][17];
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; wsel = w; }
      }
      const bool none = (bi == NOIDX);
      const int p = none ? qrow : bi;
      S pv[16];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) pv[cc] = none ? qbuf[par][cc] : cand[par][wsel][cc];
      if (p != qrow) {
        const int po = (p - j0) & 255, ps = (p - j0) >> 8;
        if (t == c2) {
#pragma unroll
          for (int cc = 0; cc < 16; ++cc) pr[0][cc] = pv[cc];
        }
        if (t == po) {
#pragma unroll
          for (int h = 0; h < H; ++h)
            if (h == ps) {
#pragma unroll
              for (int cc = 0; cc < 16; ++cc) pr[h][cc] = qbuf[par][cc];
            }
        }
      }
      const S d = pv[c2];
      if (d != (S)0) {
        const S rd = (S)1 / d;
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const int r = j0 + t + 256 * h;
          if (r > qrow && r < np) {
            const S l = pr[h][c2] * rd;
            pr[h][c2] = l;
#pragma unroll
            for (int cc = c2 + 1; cc < 16; ++cc) pr[h][cc] = fma(-l, pv[cc], pr[h][cc]);
          }
        }
      } else if (t == 0) {
        atomicOr(&plan[ii].status, 1);
        atomicMin(&plan[ii].bad_shift, k);
      }
      if (t == 0) {
        ipiv_s[c2] = p;
        ipiv[qrow] = p;
        if (p != qrow) anyswap_s = 1;
      }
    }
    // write the factored panel back, keep a copy in LDS
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int r = j0 + t + 256 * h;
      if (r < np) {
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
          W[r + (int64_t)(j0 + cc) * np] = pr[h][cc];
          panel[(r - j0) + cc * LDP] = pr[h][cc];
        }
      }
    }
    __syncthreads();

    // row interchanges outside the panel, then U12 = L11^{-1} A12
    bool sw = false;
#pragma unroll
    for (int c2 = 0; c2 < 16; ++c2) sw |= (ipiv_s[c2] != j0 + c2);
    for (int col = t; col < np; col += 256) {
      if (col >= j0 && col < j0 + 16) continue;
      S *Wc = W + (int64_t)col * np;
      if (sw) {
        for (int c2 = 0; c2 < 16; ++c2) {
          const int p = ipiv_s[c2];
          if (p != j0 + c2) {
            const S a = Wc[j0 + c2];
            Wc[j0 + c2] = Wc[p];
            Wc[p] = a;
          }
        }
      }
      if (col >= j0 + 16) {
        S u[16];
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) u[cc] = Wc[j0 + cc];
#pragma unroll
        for (int a = 0; a < 16; ++a)
#pragma unroll
          for (int b = a + 1; b < 16; ++b) u[b] = fma(-panel[b + a * LDP], u[a], u[b]);
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
          Wc[j0 + cc] = u[cc];
          u12[cc * LDU + (col - j0 - 16)] = u[cc];
        }
      }
    }
    __syncthreads();

    // trailing update A22 -= L21 U12, eight 16x16 tiles in flight per wave
    constexpr int TB = 8;
    const int nt = (np - j0 - 16) >> 4;
    const int ntt = nt * nt;
    for (int base = wave; base < ntt; base += 4 * TB) {
      v4 acc[TB];
      int tr[TB], tc[TB];
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int tile = base + 4 * u;
        tr[u] = tile % nt;
        tc[u] = tile / nt;
        if (tile < ntt)
          acc[u] = *reinterpret_cast<const v4 *>(W + (int64_t)(j0 + 16 + 16 * tc[u] + i16) * np + j0 +
                                                  16 + 16 * tr[u] + 4 * g);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          if (base + 4 * u < ntt) {
            const S a = panel[(16 + 16 * tr[u] + ar) + (4 * q + g) * LDP];
            const S b = u12[(4 * q + g) * LDU + 16 * tc[u] + i16];
            acc[u] = mfma16(-a, b, acc[u]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TB; ++u)
        if (base + 4 * u < ntt)
          *reinterpret_cast<v4 *>(W + (int64_t)(j0 + 16 + 16 * tc[u] + i16) * np + j0 + 16 +
                                   16 * tr[u] + 4 * g) = acc[u];
    }
    __syncthreads();
  }

  // 3. Permutation and inverted diagonal blocks.
  if (!anyswap_s) {
    for (int r = t; r < np; r += 256) perm[r] = r;
  } else if (t == 0) {
    for (int r = 0; r < np; ++r) perm[r] = r;
    for (int r = 0; r < np; ++r) {
      const int p = ipiv[r];
      const int a = perm[r];
      perm[r] = perm[p];
      perm[p] = a;
    }
  }
  for (int idx = t; idx < nblk * 16; idx += 256) {
    const int b = idx >> 4, j = idx & 15;
    const S *Wb = W + (int64_t)(16 * b) * np + 16 * b;
    S x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = (r == j) ? (S)1 : (S)0;
#pragma unroll
    for (int a = 0; a < 16; ++a)
#pragma unroll
      for (int r = a + 1; r < 16; ++r) x[r] = fma(-Wb[r + (int64_t)a * np], x[a], x[r]);
#pragma unroll
    for (int r = 0; r < 16; ++r) dL[b * 256 + r + 16 * j] = x[r];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = (r == j) ? (S)1 : (S)0;
#pragma unroll
    for (int a = 15; a >= 0; --a) {
      x[a] = x[a] / Wb[a + (int64_t)a * np];
#pragma unroll
      for (int r = 0; r < a; ++r) x[r] = fma(-Wb[r + (int64_t)a * np], x[a], x[r]);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) dU[b * 256 + r + 16 * j] = x[r];
  }
  __syncthreads();

  // 4. Off-diagonal blocks times the inverse of their column's diagonal block.
  {
    constexpr int TB = 4;
    const int nb2 = nblk * nblk;
    for (int base = wave; base < nb2; base += 4 * TB) {
      v4 acc[TB];
      int bi[TB], bj[TB];
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int id = base + 4 * u;
        bi[u] = id % nblk;
        bj[u] = id / nblk;
        acc[u] = MT<S>::zero();
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          if (base + 4 * u < nb2 && bi[u] != bj[u]) {
            const S a = W[(16 * bi[u] + ar) + (int64_t)(16 * bj[u] + 4 * q + g) * np];
            const S *inv = (bi[u] > bj[u] ? dL : dU) + bj[u] * 256;
            acc[u] = mfma16(a, inv[(4 * q + g) + 16 * i16], acc[u]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TB; ++u)
        if (base + 4 * u < nb2 && bi[u] != bj[u])
          *reinterpret_cast<v4 *>(W + (int64_t)(16 * bj[u] + i16) * np + 16 * bi[u] + 4 * g) = acc[u];
    }
  }
}

}  // namespace pfm
