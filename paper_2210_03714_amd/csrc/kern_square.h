// Undoing the scaling (§1): s squarings R <- R R, preceded for phi1 by the
// doubling step Phi <- (R + I) Phi / 2, which uses R before it is squared
// (phi1(2B) = (e^B + I) phi1(B) / 2).
//
// Every instance has its own s.  Level j (j = 1..max s) is one launch over
// the 64 x 64 output tiles of the instances with s >= j; the host builds the
// task list from the plan it read back, ordering it so that all tiles of one
// instance land on one XCD (workgroup b runs on XCD b mod 8) and share its L2.
// Buffers ping-pong: level j reads buffer (j-1) mod 2 and writes j mod 2.
// Stream order separates the levels, so no workgroup ever waits on another.
// Embedded (complex) instances store only the first block column
// [Re R; Im R] of emb(R); the A operand's other block column is rebuilt on
// load, emb(R)[:, hn + j] = J emb(R)[:, j], and only hn columns are produced.
#pragma once
#include "kern_common.h"

namespace pfm {

struct SqTask {
  int32_t inst;  // -1: padding
  int32_t tile;  // tile index; + (1 << 20) for the Phi product
};

// MODE 0: squaring level `level` as described above.
// MODE 1: the combination's product for the Gauss-Jordan path,
//         R = a0 I + S B (S in buffer 1, B = A 2^-s read from the caller's
//         row-major A), written to buffer 0 (and the same for Phi).
template <int MODE>
__global__ void __launch_bounds__(256)
square_level_f64_kernel(const InstDesc *__restrict__ inst, const SqTask *__restrict__ tasks,
                        int ntasks, int level, double *__restrict__ wsd,
                        const PlanRec *__restrict__ plan, double a0e, double a0p) {
  constexpr int LDA = 80, LDB = 80;  // == 16 mod 32 doubles: conflict-free fragment reads
  __shared__ double As[16 * LDA];
  __shared__ double Bs[16 * LDB];
  const int q = blockIdx.x;
  if (q >= ntasks) return;
  const SqTask tk = tasks[q];
  if (tk.inst < 0) return;
  const InstDesc D = inst[tk.inst];
  const int np = D.npad, nr = D.n, ncol = D.ncol, hn = D.hn, emb = D.emb;
  const int which = tk.tile >> 20;
  const int lt = tk.tile & ((1 << 20) - 1);
  const int tl = (np + kSqTile - 1) / kSqTile;
  const int m0 = (lt % tl) * kSqTile, n0 = (lt / tl) * kSqTile;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int ar = arow(i16);
  const int wm = wave & 1, wn = wave >> 1;

  double *base = wsd + D.r_off;
  const int64_t nn = (int64_t)np * np;
  const double *Asrc, *Bsrc;
  double *Cdst;
  int sdiv = 0;
  if (MODE == 0) {
    Asrc = base + ((level - 1) & 1) * nn;   // R_{j-1}
    Bsrc = which ? base + (2 + ((level - 1) & 1)) * nn : Asrc;
    Cdst = which ? base + (2 + (level & 1)) * nn : base + (level & 1) * nn;
  } else {
    Asrc = base + (which ? 3 : 1) * nn;     // S_e or S_p
    Bsrc = nullptr;
    Cdst = base + (which ? 2 : 0) * nn;
    sdiv = plan[tk.inst].s;
  }

  // per-thread staging: A tile 64x16 (4 consecutive rows of one k column),
  // B tile 16x64 (4 consecutive k of one column)
  const int ak = t >> 4, ar0 = (t & 15) * 4;
  const int bc = t >> 2, bk0 = (t & 3) * 4;
  double ra[4], rbv[4];
  // MODE 1 reads B row-major: 4 consecutive columns of one row per thread
  const int bk1 = t >> 4, bc1 = (t & 15) * 4;
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = m0 + ar0 + u, kc = k0 + ak;
      double a = 0.0;
      if (MODE == 1) {
        a = (r < np) ? Asrc[r + (int64_t)kc * np] : 0.0;
      } else if (r < nr && kc < nr) {
        if (!emb || kc < hn)
          a = Asrc[r + (int64_t)kc * np];
        else
          a = r < hn ? -Asrc[(r + hn) + (int64_t)(kc - hn) * np] : Asrc[(r - hn) + (int64_t)(kc - hn) * np];
      }
      if (MODE == 0 && which && r == kc) a += 1.0;  // (R + I) for the phi1 doubling
      ra[u] = a;
      if (MODE == 0) {
        const int c = n0 + bc;
        rbv[u] = (c < ncol) ? Bsrc[(k0 + bk0 + u) + (int64_t)c * np] : 0.0;
      } else {
        const int kr = k0 + bk1, c = n0 + bc1 + u;
        rbv[u] = (kr < nr && c < nr) ? ldexp(D.A[(int64_t)kr * D.lda + c], -sdiv) : 0.0;
      }
    }
  };

  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = zero4();

  load(0);
  for (int k0 = 0; k0 < np; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[ar0 + u + ak * LDA] = ra[u];
      if (MODE == 0) Bs[(bk0 + u) * LDB + bc] = rbv[u];
      else Bs[bk1 * LDB + bc1 + u] = rbv[u];
    }
    __syncthreads();
    if (k0 + 16 < np) load(k0 + 16);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[(32 * wm + 16 * a + ar) + (4 * qq + g) * LDA];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[(4 * qq + g) * LDB + 32 * wn + 16 * b + i16];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  const double scl = (MODE == 0 && which) ? 0.5 : 1.0;
  const double dia = MODE == 1 ? (which ? a0p : a0e) : 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int c = n0 + 32 * wn + 16 * b + i16;
      const int r = m0 + 32 * wm + 16 * a + 4 * g;
      if (c < ncol && r < np) {
        v4d o = acc[a][b] * scl;
        if (MODE == 1) {
#pragma unroll
          for (int v = 0; v < 4; ++v) o[v] += (r + v == c) ? dia : 0.0;
        }
        *reinterpret_cast<v4d *>(Cdst + r + (int64_t)c * np) = o;
      }
    }
}

}  // namespace pfm
