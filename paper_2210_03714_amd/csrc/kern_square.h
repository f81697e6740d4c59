// Undoing the scaling (§1): s squarings R <- R R, preceded for phi1 by the
// doubling step Phi <- (R + I) Phi / 2, which uses R before it is squared
// (phi1(2B) = (e^B + I) phi1(B) / 2), and for phi2 by
// Phi2 <- (Phi Phi + 2 Phi2) / 4 with Phi before its own step
// (phi2(2z) = (phi1(z)^2 + 2 phi2(z)) / 4, from e^{2z} - 1 - 2z =
// z^2 phi1(z)^2 + 2 z^2 phi2(z)).
//
// Every instance has its own s.  Level j (j = 1..max s) is one launch per
// tile size over the output tiles of the instances with s >= j (128 x 128
// tiles for npad >= 256, 64 x 64 below: each wave owns a (TILE/2)^2 block of
// 16 x 16 MFMA tiles, so the larger tile does 16 MFMAs per 8 LDS reads and
// 64 MFMAs between barriers); the host builds the
// task list from the plan it read back, ordering it so that all tiles of one
// instance land on one XCD (workgroup b runs on XCD b mod 8) and share its L2.
// Buffers ping-pong: level j reads buffer (j-1) mod 2 and writes j mod 2.
// Stream order separates the levels, so no workgroup ever waits on another.
// Embedded (complex) instances store only the first block column
// [Re R; Im R] of emb(R); the A operand's other block column is rebuilt on
// load, emb(R)[:, hn + j] = J emb(R)[:, j], and only hn columns are produced.
#pragma once
#include "kern_common.h"
#include "pfm.h"

namespace pfm {

struct SqTask {
  int32_t inst;  // -1: padding
  int32_t tile;  // tile index; + (1 << 20) for the Phi product, + (2 << 20) for Phi2's
};

// Buffers of an instance (np^2 doubles each, from D.r_off): R in 0 / 1, Phi
// in 2 / 3, Phi2 in 4 / 5 (level j writes j mod 2).
// MODE 0: squaring level `level` as described above.
// MODE 1: the combination's product for the Gauss-Jordan path,
//         R = a0 I + S B (S in buffer 1, B read from the row-major A: A 2^-s,
//         or A / N when `level` is 1 (action)), written to buffer 0 (and the
//         same for Phi).  Multi-workgroup-route instances use the equivalent
//         R = a0 I + alpha1 B + (B T) B, T = sum_k w_k c_k X_k, with B T
//         from MODE 2 in the (no longer needed) factor buffer: since
//         X_k = I + c_k B X_k, sum_k w_k X_k B = alpha1 B + B T B with
//         alpha1 = sum_k w_k.  The identity parts of the X_k, whose
//         rounding the weights (sum |w_k| in the hundreds) would amplify,
//         drop out; what remains of the X_k is damped by B twice.
// MODE 2: B T for the large instances: T from buffer 1 (3), B from the
//         row-major A as in MODE 1, output in the factor buffer slot 0 (1),
//         all npad columns.
// One output tile of one product (the body shared by the per-level launches
// and the persistent queue of kern_sched.h).  Ends with a barrier after its
// last LDS read, so a caller may reuse the LDS right away.
template <int MODE, int TILE>
__device__ __forceinline__ void sq_tile(const InstDesc *__restrict__ inst, const SqTask tk, int level,
                                        double *__restrict__ wsd, const PlanRec *__restrict__ plan, double a0e,
                                        double a0p, double a1e, double a1p, double a0q = 0.0) {
  static_assert(TILE == 64 || TILE == 128, "tile");
  constexpr int LDA = TILE + 16, LDB = TILE + 16;  // == 16 mod 32 doubles: conflict-free fragment reads
  constexpr int NP = TILE / 64;   // staging passes per operand
  constexpr int WT = TILE / 2;    // per-wave output block
  constexpr int NT = WT / 16;     // MFMA tiles per wave and dimension
  __shared__ double As[16 * LDA];
  __shared__ double Bs[16 * LDB];
  const InstDesc D = inst[tk.inst];
  const int np = D.npad, nr = D.n, ncol = D.ncol, hn = D.hn, emb = D.emb;
  const int which = tk.tile >> 20;
  const int lt = tk.tile & ((1 << 20) - 1);
  const int tl = (np + TILE - 1) / TILE;
  const int m0 = (lt % tl) * TILE, n0 = (lt / tl) * TILE;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  const int wm = wave & 1, wn = wave >> 1;

  double *base = wsd + D.r_off;
  const int64_t nn = (int64_t)np * np;
  const double *Asrc, *Bsrc;
  double *Cdst;
  int sdiv = 0;
  const bool act = MODE != 0 && level == 1;
  const bool q1 = MODE == 1 && plan[tk.inst].route == 2;
  double *facb = wsd + D.fac_off + (which ? nn : 0);
  const double *Qold = nullptr;  // Phi2_{j-1} (MODE 0, which 2)
  if (MODE == 0) {
    if (which == 2) {
      Asrc = base + (2 + ((level - 1) & 1)) * nn;  // Phi_{j-1} Phi_{j-1}
      Bsrc = Asrc;
      Qold = base + (4 + ((level - 1) & 1)) * nn;
      Cdst = base + (4 + (level & 1)) * nn;
    } else {
      Asrc = base + ((level - 1) & 1) * nn;   // R_{j-1}
      Bsrc = which ? base + (2 + ((level - 1) & 1)) * nn : Asrc;
      Cdst = which ? base + (2 + (level & 1)) * nn : base + (level & 1) * nn;
    }
  } else if (MODE == 1) {
    Asrc = q1 ? facb : base + (2 * which + 1) * nn;  // B T, or S_e / S_p / S_p2
    Bsrc = nullptr;
    Cdst = base + 2 * which * nn;
    sdiv = plan[tk.inst].s;
  } else {
    Asrc = nullptr;
    Bsrc = base + (which ? 3 : 1) * nn;     // T_e or T_p
    Cdst = facb;
    sdiv = plan[tk.inst].s;
  }
  auto bval = [&](int r, int c) -> double {  // B = A 2^-s or A / N, zero padded
    const double a = (r < nr && c < nr) ? D.A[(int64_t)r * D.lda + c] : 0.0;
    return act ? a / (double)sdiv : ldexp(a, -sdiv);
  };

  // per-thread staging, in NP passes of 64 rows (A) / columns (B): A tile
  // TILE x 16 (4 consecutive rows of one k column), B tile 16 x TILE (4
  // consecutive k of one column)
  const int ak = t >> 4, ar0 = (t & 15) * 4;
  const int bc = t >> 2, bk0 = (t & 3) * 4;
  double ra[NP][4], rbv[NP][4];
  // MODE 1 reads B row-major: 4 consecutive columns of one row per thread;
  // MODE 2 reads its A operand (B) row-major: 4 consecutive k of one row
  const int bk1 = t >> 4, bc1 = (t & 15) * 4;
  const int ar2 = t >> 2, ak2 = (t & 3) * 4;
  auto load = [&](int k0) {
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
      const int mo = m0 + 64 * ps, no = n0 + 64 * ps;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = mo + ar0 + u, kc = k0 + ak;
        double a = 0.0;
        if (MODE == 2) {
          a = bval(mo + ar2, k0 + ak2 + u);
        } else if (MODE == 1) {
          a = (r < np) ? Asrc[r + (int64_t)kc * np] : 0.0;
        } else if (r < nr && kc < nr) {
          if (!emb || kc < hn)
            a = Asrc[r + (int64_t)kc * np];
          else
            a = r < hn ? -Asrc[(r + hn) + (int64_t)(kc - hn) * np] : Asrc[(r - hn) + (int64_t)(kc - hn) * np];
        }
        if (MODE == 0 && which == 1 && r == kc) a += 1.0;  // (R + I) for the phi1 doubling
        ra[ps][u] = a;
        if (MODE == 0) {
          const int c = no + bc;
          rbv[ps][u] = (c < ncol) ? Bsrc[(k0 + bk0 + u) + (int64_t)c * np] : 0.0;
        } else if (MODE == 2) {
          const int c = no + bc;
          rbv[ps][u] = (c < np) ? Bsrc[(k0 + bk0 + u) + (int64_t)c * np] : 0.0;
        } else {
          rbv[ps][u] = bval(k0 + bk1, no + bc1 + u);
        }
      }
    }
  };

  v4d acc[NT][NT];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = zero4();

  load(0);
  for (int k0 = 0; k0 < np; k0 += 16) {
#pragma unroll
    for (int ps = 0; ps < NP; ++ps)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (MODE == 2) As[64 * ps + ar2 + (ak2 + u) * LDA] = ra[ps][u];
        else As[64 * ps + ar0 + u + ak * LDA] = ra[ps][u];
        if (MODE != 1) Bs[(bk0 + u) * LDB + 64 * ps + bc] = rbv[ps][u];
        else Bs[bk1 * LDB + 64 * ps + bc1 + u] = rbv[ps][u];
      }
    __syncthreads();
    if (k0 + 16 < np) load(k0 + 16);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      double av[NT], bv[NT];
#pragma unroll
      for (int a = 0; a < NT; ++a) av[a] = As[(WT * wm + 16 * a + ar) + (4 * qq + g) * LDA];
#pragma unroll
      for (int b = 0; b < NT; ++b) bv[b] = Bs[(4 * qq + g) * LDB + WT * wn + 16 * b + i16];
#pragma unroll
      for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  const double scl = MODE == 0 ? (which == 2 ? 0.25 : (which ? 0.5 : 1.0)) : 1.0;
  const double dia = MODE == 1 ? (which == 2 ? a0q : (which ? a0p : a0e)) : 0.0;
  const double lin = q1 ? (which ? a1p : a1e) : 0.0;
  const int oc = MODE == 2 ? np : ncol;  // computed columns
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const int c = n0 + WT * wn + 16 * b + i16;
      const int r = m0 + WT * wm + 16 * a + 4 * g;
      if (c < oc && r < np) {
        v4d o = acc[a][b] * scl;
        if (MODE == 0 && which == 2) {
          const v4d q = *reinterpret_cast<const v4d *>(Qold + r + (int64_t)c * np);
#pragma unroll
          for (int v = 0; v < 4; ++v) o[v] = fma(0.5, q[v], o[v]);
        }
        if (MODE == 1) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            o[v] += (r + v == c) ? dia : 0.0;
            if (q1) o[v] = fma(lin, bval(r + v, c), o[v]);
          }
        }
        *reinterpret_cast<v4d *>(Cdst + r + (int64_t)c * np) = o;
      }
    }
}

// One launch over a task list.  Every candidate instance is listed (the host
// does not know the plans): MODE 0 tasks of instances with s < level, and
// MODE 1 / 2 tasks of instances on another route, return at once.
template <int MODE, int TILE>
__global__ void __launch_bounds__(256, 2)
square_level_f64_kernel(const InstDesc *__restrict__ inst, const SqTask *__restrict__ tasks,
                        int ntasks, int level, double *__restrict__ wsd,
                        const PlanRec *__restrict__ plan, double a0e, double a0p,
                        double a1e = 0.0, double a1p = 0.0, double a0q = 0.0) {
  const int q = blockIdx.x;
  if (q >= ntasks) return;
  const SqTask tk = tasks[q];
  if (tk.inst < 0) return;
  const PlanRec &P = plan[tk.inst];
  if (P.status & PFM_NOT_COMPUTED) return;
  if (MODE == 0 && P.s < level) return;
  if (MODE == 1 && P.route == 0) return;
  if (MODE == 2 && P.route != 2) return;
  sq_tile<MODE, TILE>(inst, tk, level, wsd, plan, a0e, a0p, a1e, a1p, a0q);
}

}  // namespace pfm
