// Large instances (npad > 512, real or embedded complex): the shifted
// inverses X_k = (I - c_k B)^{-1} by block Gauss-Jordan spread over many
// workgroups, then the action steps as skinny GEMMs with the explicit r(B).
//
// The host sends an instance here only when |c_k| ||M||_1 <= 1/2 for the
// real matrix M the kernels see (B, or emb(B) with ||emb(B)||_1 <=
// sqrt(2) ||B||_1), so every I - c_k M is strictly column diagonally dominant
// and Gauss-Jordan without interchanges is what partial pivoting would do.
//
// Block step J (64-column blocks, W column-major npad x npad per shift):
//   ln_dinv_kernel (one workgroup per (instance, shift)):
//       Dinv = D^{-1}, D = W[J, J] taken from colbuf (the column block J as
//       it was before the step), into the dinv buffer.
//   ln_row_kernel  (one workgroup per column block C):
//       C == J: W[J, J] <- Dinv;
//       C != J: W[J, C] <- Dinv W[J, C]; for C == J + 1 also into the next
//       colbuf.
//   ln_upd_kernel  (one workgroup per 128 rows x column block C):
//       C != J: W[I, C] <- W[I, C] - colbuf[I] W[J, C]   (new row block)
//       C == J: W[I, J] <- -colbuf[I] Dinv
//       rows I outside block J; C == J + 1 also into the next colbuf.
// colbuf ping-pongs between steps, so no launch reads what it overwrites.
#pragma once
#include "kern_common.h"

namespace pfm {

constexpr int kLB = 64;     // Gauss-Jordan block width
constexpr int kLRows = 128; // rows per update workgroup (4 waves x 32)
constexpr int kLKC = 256;   // K chunk of the action-step GEMM (npad > 1024)

// per-shift side buffers: colbuf[2] (npad x 64 column-major each), dinv (64 x 64)
__host__ __device__ inline int64_t ln_stride(int np) { return 2 * (int64_t)np * kLB + kLB * kLB; }

// W_k = I - c_k B column-major, B = A 2^-s (full) or A / N (action), from the
// row-major A (the embedded matrix for complex instances); tiles of column
// block 0 also go to colbuf[0].  Grid: xcd over (instance, shift) slots x
// 64 x 64 tiles.
__global__ void __launch_bounds__(256)
ln_load_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nslot,
               int ntile1, const PlanRec *__restrict__ plan, Terms T, double *__restrict__ wsd,
               int action) {
  __shared__ double tile[kLB][kLB + 1];
  int slot, sub;
  xcd_map(blockIdx.x, ntile1 * ntile1, slot, sub);
  if (slot >= nslot) return;
  const int li = slot / T.nterms, k = slot % T.nterms;
  const int ii = ilist[li];
  if (!on_route(plan[ii], 2)) return;
  const InstDesc D = inst[ii];
  const int n = D.n, np = D.npad;
  const int tr = sub % ntile1, tc = sub / ntile1;
  if (tr * kLB >= np || tc * kLB >= np) return;
  const int t = threadIdx.x;
  const double c = T.c_re[k];
  const int sN = plan[ii].s;
  const double cs = ldexp(c, -sN);
  const double Nd = (double)sN;
  const int r0 = tr * kLB, c0 = tc * kLB;
  {
    const int cc = t & 63;
#pragma unroll 4
    for (int u = 0; u < 16; ++u) {
      const int rr = (t >> 6) + 4 * u;
      const int r = r0 + rr, col = c0 + cc;
      tile[rr][cc] = (r < n && col < n) ? D.A[(int64_t)r * D.lda + col] : 0.0;
    }
  }
  __syncthreads();
  double *W = wsd + D.fac_off + (int64_t)k * np * np;
  double *cb0 = wsd + D.ln_off + (int64_t)k * ln_stride(np);
  const int rr = t & 63;
#pragma unroll 4
  for (int u = 0; u < 16; ++u) {
    const int cc = (t >> 6) + 4 * u;
    const int r = r0 + rr, col = c0 + cc;
    const double a = tile[rr][cc];
    const double cb = action ? c * (a / Nd) : cs * a;
    const double v = (r == col ? 1.0 : 0.0) - cb;
    W[r + (int64_t)col * np] = v;
    if (tc == 0) cb0[r + (int64_t)cc * np] = v;
  }
}

// 64 x 64 Gauss-Jordan inversion in LDS (row-major, leading dimension LDD),
// no interchanges; 256 threads, each owning a 4 x 4 patch.
template <int LDD>
__device__ __forceinline__ void ln_gj64(double *Dl, int pr0, int pc0) {
#pragma unroll 1
  for (int c = 0; c < kLB; ++c) {
    const double p = 1.0 / Dl[c * LDD + c];
    double colc[4], rowc[4], cur[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) colc[a] = Dl[(pr0 + a) * LDD + c];
#pragma unroll
    for (int b = 0; b < 4; ++b) rowc[b] = Dl[c * LDD + pc0 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) cur[a][b] = Dl[(pr0 + a) * LDD + pc0 + b];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = pr0 + a;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = pc0 + b;
        double v;
        if (i == c && j == c) v = p;
        else if (i == c) v = rowc[b] * p;
        else if (j == c) v = -colc[a] * p;
        else v = fma(-colc[a] * p, rowc[b], cur[a][b]);
        Dl[i * LDD + j] = v;
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256)
ln_dinv_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nslot, Terms T,
               double *__restrict__ wsd, int J, const PlanRec *__restrict__ plan) {
  constexpr int LDD = kLB + 1;
  __shared__ double Dl[kLB * LDD];
  const int slot = blockIdx.x;
  if (slot >= nslot) return;
  const int li = slot / T.nterms, k = slot % T.nterms;
  if (!on_route(plan[ilist[li]], 2)) return;
  const InstDesc D = inst[ilist[li]];
  const int np = D.npad, nJ = np / kLB;
  if (J >= nJ) return;
  const int t = threadIdx.x;
  const double *side = wsd + D.ln_off + (int64_t)k * ln_stride(np);
  const double *colJ = side + (int64_t)(J & 1) * np * kLB;
  double *dinv = wsd + D.ln_off + (int64_t)k * ln_stride(np) + 2 * (int64_t)np * kLB;
  const int j0 = J * kLB;
  const int pr0 = (t >> 4) * 4, pc0 = (t & 15) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Dl[(pr0 + a) * LDD + pc0 + b] = colJ[(j0 + pr0 + a) + (int64_t)(pc0 + b) * np];
  __syncthreads();
  ln_gj64<LDD>(Dl, pr0, pc0);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) dinv[(pr0 + a) + (pc0 + b) * kLB] = Dl[(pr0 + a) * LDD + pc0 + b];
}

__global__ void __launch_bounds__(256)
ln_row_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nslot, int nJmax,
              Terms T, double *__restrict__ wsd, int J, const PlanRec *__restrict__ plan) {
  constexpr int LDD = kLB + 1;
  __shared__ double Dl[kLB * LDD];
  __shared__ double Cl[kLB * LDD];
  int slot, C;
  xcd_map(blockIdx.x, nJmax, slot, C);
  if (slot >= nslot) return;
  const int li = slot / T.nterms, k = slot % T.nterms;
  if (!on_route(plan[ilist[li]], 2)) return;
  const InstDesc D = inst[ilist[li]];
  const int np = D.npad, nJ = np / kLB;
  if (J >= nJ || C >= nJ) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  double *W = wsd + D.fac_off + (int64_t)k * np * np;
  double *side = wsd + D.ln_off + (int64_t)k * ln_stride(np);
  double *colN = side + (int64_t)((J + 1) & 1) * np * kLB;
  const double *dinv = side + 2 * (int64_t)np * kLB;
  const int j0 = J * kLB, c0 = C * kLB;
  const int pr0 = (t >> 4) * 4, pc0 = (t & 15) * 4;
  if (C == J) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        W[(j0 + pr0 + a) + (int64_t)(j0 + pc0 + b) * np] = dinv[(pr0 + a) + (pc0 + b) * kLB];
    return;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      Dl[(pr0 + a) * LDD + pc0 + b] = dinv[(pr0 + a) + (pc0 + b) * kLB];
      Cl[(pr0 + a) * LDD + pc0 + b] = W[(j0 + pr0 + a) + (int64_t)(c0 + pc0 + b) * np];
    }
  __syncthreads();
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = zero4();
#pragma unroll 4
  for (int q = 0; q < kLB / 4; ++q) {
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
    for (int b = 0; b < 2; ++b) {
      const int rr = wr + 16 * a + 4 * g, cc = wc + 16 * b + i16;
      *reinterpret_cast<v4d *>(W + (j0 + rr) + (int64_t)(c0 + cc) * np) = acc[a][b];
      if (C == J + 1) *reinterpret_cast<v4d *>(colN + (j0 + rr) + (int64_t)cc * np) = acc[a][b];
    }
}

__global__ void __launch_bounds__(256)
ln_upd_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nslot, int nJmax,
              int nRmax, Terms T, double *__restrict__ wsd, int J, const PlanRec *__restrict__ plan) {
  constexpr int LDB = 80;  // == 16 mod 32 doubles
  __shared__ double Bl[kLB * LDB];
  int slot, sub;
  xcd_map(blockIdx.x, nJmax * nRmax, slot, sub);
  if (slot >= nslot) return;
  const int C = sub / nRmax, rc = sub % nRmax;
  const int li = slot / T.nterms, k = slot % T.nterms;
  if (!on_route(plan[ilist[li]], 2)) return;
  const InstDesc D = inst[ilist[li]];
  const int np = D.npad, nJ = np / kLB;
  if (J >= nJ || C >= nJ || rc * kLRows >= np) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  double *W = wsd + D.fac_off + (int64_t)k * np * np;
  double *side = wsd + D.ln_off + (int64_t)k * ln_stride(np);
  const double *colJ = side + (int64_t)(J & 1) * np * kLB;
  double *colN = side + (int64_t)((J + 1) & 1) * np * kLB;
  const double *dinv = side + 2 * (int64_t)np * kLB;
  const int j0 = J * kLB, c0 = C * kLB;
  // B operand: the new row block W[J, C] (C != J) or Dinv (C == J), row-major in LDS
  {
    const int cc = t & 63;
#pragma unroll 4
    for (int u = 0; u < 16; ++u) {
      const int kr = (t >> 6) + 4 * u;
      Bl[kr * LDB + cc] = C == J ? dinv[kr + cc * kLB] : W[(j0 + kr) + (int64_t)(c0 + cc) * np];
    }
  }
  __syncthreads();
  const int r0 = rc * kLRows + 32 * wave;
  if (r0 >= np || (r0 >= j0 && r0 < j0 + kLB)) return;  // no barrier follows
  v4d acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      acc[a][b] = C == J ? zero4()
                         : *reinterpret_cast<const v4d *>(W + (r0 + 16 * a + 4 * g) + (int64_t)(c0 + 16 * b + i16) * np);
#pragma unroll 4
  for (int q = 0; q < kLB / 4; ++q) {
    const int kk = 4 * q + g;
    double av[2], bv[4];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = -colJ[(r0 + 16 * a + ar) + (int64_t)kk * np];
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = Bl[kk * LDB + 16 * b + i16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int rr = r0 + 16 * a + 4 * g, cc = 16 * b + i16;
      *reinterpret_cast<v4d *>(W + rr + (int64_t)(c0 + cc) * np) = acc[a][b];
      if (C == J + 1) *reinterpret_cast<v4d *>(colN + rr + (int64_t)cc * np) = acc[a][b];
    }
}

// ---------------------------------------------------------------------------
// Action steps with the explicit approximant.  M (R = r(B) in R buffer 0, or
// the phi1 approximant P in buffer 2) is stored column-major npad x ncol; an
// embedded instance stores only the first block column [Re; Im] and the
// second is rebuilt on load as J times the first.  Vectors U are row-major
// npad x pp (pp = p rounded up to 16); embedded: rows [Re; Im].
//
// Per chain (exp, or phi1) and instance, at D.v_off:
//   U[2] (ping-pong), U1 (phi1: the first iterate), then the K-split
//   partial products part[KS] (shared by the chains, which run in turn).

__host__ __device__ inline int ln_pp(int p) { return (p + 15) / 16 * 16; }
__host__ __device__ inline int ln_ks(int n) { return (n + kLKC - 1) / kLKC; }
__host__ __device__ inline int64_t ln_vchain(int np, int p) { return 3 * (int64_t)np * ln_pp(p); }

// U[0] of each chain <- V (zero padded).  Grid: x = 64-row chunk, y = instance in list.
__global__ void __launch_bounds__(256)
ln_vprep_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nchain,
                double *__restrict__ wsd, const PlanRec *__restrict__ plan) {
  if (!on_route(plan[ilist[blockIdx.y]], 2)) return;
  const InstDesc D = inst[ilist[blockIdx.y]];
  const int np = D.npad, pp = ln_pp(D.p);
  const int r0 = blockIdx.x * 64;
  if (r0 >= np) return;
  for (int e = threadIdx.x; e < 64 * pp; e += 256) {
    const int r = r0 + e / pp, c = e % pp;
    double v = 0.0;
    if (c < D.p) {
      if (!D.emb) {
        if (r < D.n) v = D.V[(int64_t)r * D.ldv + c];
      } else if (r < D.n) {
        const int rr = r < D.hn ? r : r - D.hn;
        v = D.cin ? D.V[2 * ((int64_t)rr * D.ldv + c) + (r < D.hn ? 0 : 1)] : (r < D.hn ? D.V[(int64_t)rr * D.ldv + c] : 0.0);
      }
    }
    for (int ch = 0; ch < nchain; ++ch) wsd[D.v_off + ch * ln_vchain(np, D.p) + (int64_t)r * pp + c] = v;
  }
}

// part[ks] = M[:, K chunk ks] U_in[K chunk ks, :].  Grid: xcd over list
// entries x (row tiles of 64 x K chunks).  Instances with N < step skip.
template <int PP>
__global__ void __launch_bounds__(256)
ln_gemv_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nl, int nsub,
               const PlanRec *__restrict__ plan, double *__restrict__ wsd, int step, int chain,
               int use_p, int in_buf) {
  int slot, sub;
  xcd_map(blockIdx.x, nsub, slot, sub);
  if (slot >= nl) return;
  const int ii = ilist[slot];
  if (!on_route(plan[ii], 2)) return;
  const InstDesc D = inst[ii];
  if (step > plan[ii].s) return;
  const int np = D.npad, nr = D.n, hn = D.hn, emb = D.emb;
  if (ln_pp(D.p) != PP) return;  // never sent
  const int ntr = np / 64, KS = ln_ks(nr);
  const int rt = sub % ntr, ks = sub / ntr;
  if (ks >= KS) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  const double *M = wsd + D.r_off + (use_p ? 2 : 0) * (int64_t)np * np;
  const double *U = wsd + D.v_off + chain * ln_vchain(np, D.p) + (int64_t)in_buf * np * PP;
  double *part = wsd + D.v_off + 2 * ln_vchain(np, D.p) + (int64_t)ks * np * PP;
  const int r = rt * 64 + 16 * wave + ar;
  const int kb = ks * kLKC, ke = min(nr, kb + kLKC);
  v4d acc[PP / 16];
#pragma unroll
  for (int b = 0; b < PP / 16; ++b) acc[b] = zero4();
#pragma unroll 4
  for (int k0 = kb; k0 < ke; k0 += 4) {
    const int kc = k0 + g;
    double a = 0.0;
    if (r < nr && kc < ke) {
      if (!emb || kc < hn) a = M[r + (int64_t)kc * np];
      else a = r < hn ? -M[(r + hn) + (int64_t)(kc - hn) * np] : M[(r - hn) + (int64_t)(kc - hn) * np];
    }
#pragma unroll
    for (int b = 0; b < PP / 16; ++b) {
      const double bv = kc < ke ? U[(int64_t)kc * PP + 16 * b + i16] : 0.0;
      acc[b] = mfma16(a, bv, acc[b]);
    }
  }
  const int ro = rt * 64 + 16 * wave + 4 * g;
#pragma unroll
  for (int b = 0; b < PP / 16; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) part[(int64_t)(ro + v) * PP + 16 * b + i16] = acc[b][v];
}

// U_out = scale * sum_ks part[ks] (+ U1); set_u1 keeps the result as U1; on
// the instance's last step the result goes to the caller's output (row-major
// n x p; complex interleaved for complex instances).  Grid: x = 64-row chunk,
// y = instance in list.
__global__ void __launch_bounds__(256)
ln_vreduce_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist,
                  const PlanRec *__restrict__ plan, double *__restrict__ wsd, int step, int chain,
                  int out_buf, double scale_first, int phi) {
  const int ii = ilist[blockIdx.y];
  if (!on_route(plan[ii], 2)) return;
  const InstDesc D = inst[ii];
  const int N = plan[ii].s;
  if (step > N) return;
  const int np = D.npad, pp = ln_pp(D.p), KS = ln_ks(D.n);
  const int r0 = blockIdx.x * 64;
  if (r0 >= np) return;
  double *base = wsd + D.v_off + chain * ln_vchain(np, D.p);
  double *Uo = base + (int64_t)out_buf * np * pp;
  double *U1 = base + 2 * (int64_t)np * pp;
  const double *part = wsd + D.v_off + 2 * ln_vchain(np, D.p);
  const double scale = (phi && step == 1) ? 1.0 / (double)N : scale_first;
  double *F = phi ? D.Fp : D.Fe;
  for (int e = threadIdx.x; e < 64 * pp; e += 256) {
    const int r = r0 + e / pp, c = e % pp;
    const int64_t o = (int64_t)r * pp + c;
    double v = 0.0;
    for (int ks = 0; ks < KS; ++ks) v += part[(int64_t)ks * np * pp + o];
    v *= scale;
    if (phi) {
      if (step == 1) U1[o] = v;
      else v += U1[o];
    }
    Uo[o] = v;
    if (step == N && c < D.p && r < D.n) {
      if (!D.emb) {
        F[(int64_t)r * D.ldf + c] = v;
      } else {
        const int rr = r < D.hn ? r : r - D.hn;
        F[2 * ((int64_t)rr * D.ldf + c) + (r < D.hn ? 0 : 1)] = v;
      }
    }
  }
}

// All N steps of the action for one (instance, function, 16-column slab)
// in one workgroup, for npad <= NPMAX <= 512: U (npad x 16) lives in LDS;
// each wave computes its 16-row tiles of M U (M = R, or the phi1
// approximant P on the phi1 chain's first step, scaled by 1/N) into
// registers, then after a barrier writes them back into U; the phi1 chain
// keeps u_1 in the instance's workspace (each thread rereads only what it
// wrote) and adds it every later step.  Only barriers inside
// the workgroup; M is read from memory every step (L2 / MALL).  The result
// goes to the caller's output (row-major n x p; complex interleaved).
// Grid: xcd over list entries x (chains x slabs).
template <int NPMAX>
__global__ void __launch_bounds__(256, 1)
ln_steps_kernel(const InstDesc *__restrict__ inst, const int *__restrict__ ilist, int nl, int nslab,
                const PlanRec *__restrict__ plan, double *__restrict__ wsd, int want_exp,
                int want_phi) {
  constexpr int RT = NPMAX / 64;  // 16-row tiles per wave
  __shared__ double Us[NPMAX * 16];
  const int nchain = want_exp + want_phi;
  int slot, sub;
  xcd_map(blockIdx.x, nchain * nslab, slot, sub);
  if (slot >= nl) return;
  const int ch = sub / nslab, slab = sub % nslab;
  const bool phi = ch == 1 || !want_exp;
  const int ii = ilist[slot];
  if (!on_route(plan[ii], 2)) return;
  const InstDesc D = inst[ii];
  const int np = D.npad, nr = D.n, hn = D.hn, emb = D.emb, p = D.p;
  const int c0 = slab * 16;
  if (np > NPMAX || c0 >= p) return;  // uniform over the workgroup
  const int N = plan[ii].s;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  const double *Rm = wsd + D.r_off;
  const double *Pm = Rm + 2 * (int64_t)np * np;
  const int pp = ln_pp(p);
  double *U1 = wsd + D.v_off + ch * ln_vchain(np, p) + 2 * (int64_t)np * pp;  // row-major np x pp

  for (int e = t; e < np * 16; e += 256) {  // U = V[:, slab] (real: rows < n; emb: [Re; Im])
    const int r = e >> 4, c = c0 + (e & 15);
    double v = 0.0;
    if (c < p && r < nr) {
      if (!emb) {
        v = D.V[(int64_t)r * D.ldv + c];
      } else {
        const int rr = r < hn ? r : r - hn;
        v = D.cin ? D.V[2 * ((int64_t)rr * D.ldv + c) + (r < hn ? 0 : 1)] : (r < hn ? D.V[(int64_t)rr * D.ldv + c] : 0.0);
      }
    }
    Us[e] = v;
  }
  __syncthreads();

  constexpr int RTP = RT < 4 ? RT : 4;  // tiles per pass (register budget)
  constexpr int NPASS = RT / RTP;
#pragma unroll 1
  for (int j = 1; j <= N; ++j) {
    const double *M = (phi && j == 1) ? Pm : Rm;
    double *Un = wsd + D.v_off + ch * ln_vchain(np, p) + (int64_t)(j & 1) * np * pp;  // new U (row-major)
#pragma unroll 1
    for (int pass = 0; pass < NPASS; ++pass) {
      v4d acc[RTP];
#pragma unroll
      for (int rt = 0; rt < RTP; ++rt) acc[rt] = zero4();
#pragma unroll 2
      for (int k0 = 0; k0 < nr; k0 += 4) {
        const int kc = k0 + g;
        const double b = kc < nr ? Us[kc * 16 + i16] : 0.0;
#pragma unroll
        for (int rt = 0; rt < RTP; ++rt) {
          const int r = (wave + 4 * (pass * RTP + rt)) * 16 + ar;
          double a = 0.0;
          if (r < nr && kc < nr) {
            if (!emb || kc < hn) a = M[r + (int64_t)kc * np];
            else a = r < hn ? -M[(r + hn) + (int64_t)(kc - hn) * np] : M[(r - hn) + (int64_t)(kc - hn) * np];
          }
          acc[rt] = mfma16(a, b, acc[rt]);
        }
      }
#pragma unroll
      for (int rt = 0; rt < RTP; ++rt) {
        const int r = (wave + 4 * (pass * RTP + rt)) * 16 + 4 * g;
        if (r >= np) continue;
        if (phi) {
          double *u = U1 + (int64_t)r * pp + c0 + i16;
          if (j == 1) {
            acc[rt] = acc[rt] * (1.0 / (double)N);
#pragma unroll
            for (int v = 0; v < 4; ++v) u[(int64_t)v * pp] = acc[rt][v];
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[rt][v] += u[(int64_t)v * pp];
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Un[(int64_t)(r + v) * pp + c0 + i16] = acc[rt][v];
      }
    }
    __syncthreads();  // every wave has read U and written its rows of the new U
    for (int e = t; e < np * 16; e += 256) Us[e] = Un[(int64_t)(e >> 4) * pp + c0 + (e & 15)];
    __syncthreads();  // the new U is in LDS
  }
  double *F = phi ? D.Fp : D.Fe;
  for (int e = t; e < nr * 16; e += 256) {
    const int r = e >> 4, c = c0 + (e & 15);
    if (c >= p) continue;
    const double v = Us[e];
    if (!emb) {
      F[(int64_t)r * D.ldf + c] = v;
    } else {
      const int rr = r < hn ? r : r - hn;
      F[2 * ((int64_t)rr * D.ldf + c) + (r < hn ? 0 : 1)] = v;
    }
  }
}

}  // namespace pfm
