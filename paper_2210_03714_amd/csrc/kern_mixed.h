// Mixed-precision shifted solves (full-matrix path).
//
// The factors of M_k = I - c_k B are computed in binary32 (lu_kernel<.., float>,
// v_mfma_f32_16x16x4 trailing updates).  Each solve Z_k = M_k^{-1} B is then
// refined in binary64:
//   Z <- 0, r <- B
//   repeat: Z <- Z + solve32(r)                       (binary32 LU, MFMA)
//           r <- B - M Z = B - Z + c_k (B Z)          (binary64 MFMA GEMM)
//   until max|r| <= irtol max|B| or maxit sweeps,
// and the combination sum_k w_k Z_k (round-off form, §4.3) and the squarings
// stay in binary64.  irtol = tol / (4 sum_k |w_k|): the cancellation in the
// combination amplifies a solve error by at most sum |w_k|.
//
// One workgroup per (instance, column slab), as in the binary64 solve.  r and
// Z are binary64 MFMA fragments; r is permuted through LDS and rounded to
// binary32 for the correction solve; B Z takes B column-major from the
// workspace (A operand) and Z from LDS (B operand).
#pragma once
#include "kern_solve.h"

namespace pfm {

template <int NPMAX, int SW, bool PHI>
__global__ void __launch_bounds__(256, 1)
solve_mixed_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nlist,
                   PlanRec *__restrict__ plan, Terms T, double *__restrict__ wsd,
                   const int *__restrict__ wsi, int maxit, double irtol) {
  constexpr int RB = NPMAX / 64;
  constexpr int CT = SW / 16;
  constexpr int NSLAB = NPMAX / SW;
  constexpr int PRB = PHI ? RB : 1;
  __shared__ double Ybuf[NPMAX * SW];
  __shared__ float S32[2][16 * SW];
  __shared__ float Tst32[4][16 * SW];
  __shared__ double red[2][4];

  int slot, sl;
  xcd_map(blockIdx.x, NSLAB, slot, sl);
  if (slot >= nlist) return;
  const int ii = ilist[slot];
  if (!on_route(plan[ii], 0)) return;  // not computed
  const InstDesc D = inst[ii];
  const int n = D.n, np = D.npad;
  if (np > NPMAX || (np & 15) || n > np || n < 1) return;  // sizes the host never sends
  const int c0 = sl * SW;
  const int ncol = D.ncol;
  if (c0 >= ncol) return;
  const int nblk = np >> 4;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar64 = arow(i16), ar32 = MT<float>::arow_(i16);
  const double sc = ldexp(1.0, -plan[ii].s);
  const double *Bt = wsd + D.e_off;  // B = 2^-s A, column-major

  v4d Zd[RB][CT], Rd[RB][CT], Ae[RB][CT], Ap[PRB][CT];
  v4f Zf[RB][CT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) Ae[rb][ct] = zero4();
#pragma unroll
  for (int rb = 0; rb < PRB; ++rb)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) Ap[rb][ct] = zero4();

  // element (rb, ct, v) of B[:, slab] in natural row order.  The base
  // pointer is made opaque at every use, so that the addresses of these
  // loads are formed where they are used rather than held in registers
  // across the shifts (at npad = 512 that is 32 64-bit addresses a lane).
  auto b_elem = [&](const double *Ab, int rb, int ct, int v) -> double {
    const int b = wave + 4 * rb, col = c0 + 16 * ct + i16, r = 16 * b + 4 * g + v;
    return (b < nblk && r < n && col < ncol) ? sc * Ab[(int64_t)r * D.lda + col] : 0.0;
  };
  auto opaque_a = [&]() {
    const double *Ab = D.A;
    asm volatile("" : "+v"(Ab));
    return Ab;
  };
  auto load_b = [&](v4d (&X)[RB][CT]) {
    const double *Ab = opaque_a();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) X[rb][ct][v] = b_elem(Ab, rb, ct, v);
  };
  // workgroup-wide max |X| (all threads get the value)
  int par = 0;
  auto wg_max = [&](const v4d (&X)[RB][CT]) -> double {
    double m = 0.0;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) m = fmax(m, fabs(X[rb][ct][v]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane == 0) red[par][wave] = m;
    __syncthreads();
    const double r = fmax(fmax(red[par][0], red[par][1]), fmax(red[par][2], red[par][3]));
    par ^= 1;
    return r;
  };

  int it_max = 0;
  double res_max = 0.0;
#pragma unroll 1
  for (int k = 0; k < T.nterms; ++k) {
    const float *Wf = reinterpret_cast<const float *>(wsd + D.fac_off) + (int64_t)k * np * np;
    const int *perm = wsi + D.perm_ioff + (int64_t)k * np;
    const float *dL = reinterpret_cast<const float *>(wsd + D.dinv_off) + (int64_t)(2 * k) * nblk * 256;
    const float *dU = dL + (int64_t)nblk * 256;
    const double ck = T.c_re[k];

    load_b(Rd);
    const double bmax = wg_max(Rd);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) Zd[rb][ct] = zero4();

    int it = 0;
    double rrel = 1.0;
#pragma unroll 1
    for (;;) {
      // correction: Z += M^{-1} r with the binary32 factors
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int b = wave + 4 * rb;
        if (b < nblk) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) Ybuf[(16 * b + 4 * g + v) * SW + 16 * ct + i16] = Rd[rb][ct][v];
        }
      }
      __syncthreads();
      {
        const int *pk = perm;
        asm volatile("" : "+v"(pk));  // (as for B's loads)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int b = wave + 4 * rb;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              Zf[rb][ct][v] = (b < nblk) ? (float)Ybuf[pk[16 * b + 4 * g + v] * SW + 16 * ct + i16] : 0.f;
        }
      }
      __syncthreads();
      lu_solve_slab<RB, CT, SW, float>(Zf, Wf, dL, dU, S32, Tst32[wave], np, nblk, wave, ar32, g, i16);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) Zd[rb][ct][v] += (double)Zf[rb][ct][v];
      if (it == maxit) break;
      ++it;
      // residual r = B - Z + c (B Z) in binary64
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int b = wave + 4 * rb;
        if (b < nblk) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) Ybuf[(16 * b + 4 * g + v) * SW + 16 * ct + i16] = Zd[rb][ct][v];
        }
      }
      __syncthreads();
      // B Z accumulates in r's registers (r is formed again from B below)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) Rd[rb][ct] = zero4();
#pragma unroll 2
      for (int k0 = 0; k0 < np; k0 += 4) {
        double bf[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) bf[ct] = Ybuf[(k0 + g) * SW + 16 * ct + i16];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int bb = wave + 4 * rb;
          if (bb < nblk) {
            const double a = Bt[(16 * bb + ar64) + (int64_t)(k0 + g) * np];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) Rd[rb][ct] = mfma16(a, bf[ct], Rd[rb][ct]);
          }
        }
      }
      __syncthreads();
      {
        const double *Ab = opaque_a();
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              Rd[rb][ct][v] = fma(ck, Rd[rb][ct][v], b_elem(Ab, rb, ct, v) - Zd[rb][ct][v]);
      }
      const double rmax = wg_max(Rd);
      rrel = bmax > 0.0 ? rmax / bmax : 0.0;
      if (rrel <= irtol) break;
    }
    it_max = it > it_max ? it : it_max;
    res_max = fmax(res_max, rrel);

    const double we = T.we_re[k], wp = T.wp_re[k];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Ae[rb][ct][v] = fma(we, Zd[rb][ct][v], Ae[rb][ct][v]);
        if constexpr (PHI) {
#pragma unroll
          for (int v = 0; v < 4; ++v) Ap[rb][ct][v] = fma(wp, Zd[rb][ct][v], Ap[rb][ct][v]);
        }
      }
    __syncthreads();
  }
  if (t == 0) {
    atomicMax(&plan[ii].ir_iters, it_max);
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long *>(&plan[ii].resid),
              (unsigned long long)__double_as_longlong(res_max));
    if (res_max > irtol) atomicOr(&plan[ii].status, 4);
  }

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
