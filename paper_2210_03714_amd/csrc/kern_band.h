// Banded A (half-bandwidth b, 1 <= b <= kBandMaxB): the action f(A)V by the
// N-step recurrence with the round-off form of §4.3.  §2.1 and §5 name the
// pentadiagonal case (b = 2) beside the tridiagonal one: I - c_k B keeps the
// band of A, so each shifted system costs one banded forward and backward
// sweep, and the LU of every shifted matrix is formed once and reused by all
// N steps and all columns (§5.1).  With ||B||_1 <= θ every I - c_k B is
// strictly column diagonally dominant, so elimination without interchanges
// is the partial-pivoting LU.
//
// Two step kernels share the factorisation:
//   band_scan_kernel (b = 2, up to 8 shifts, d <= kTsMaxD): a wave per shift,
//     one column at a time, the sweeps as 2-state affine maps scanned over
//     the lanes, the vector in LDS for all N steps (described above the
//     kernel);
//   band_steps_kernel (the rest): a lane per column, a wave per 64
//     consecutive columns of one instance (every lane needs the same rows of
//     B and of the factors), the vector in memory between the passes of a
//     step (below).
// Layout:
//   A:        bands[(b + o) d + i] = A[i][i + o], o = -b..b (caller's; the
//             entries with i + o outside [0, d) are never read)
//   B:        row-major, B[r][r + o] at r (2b + 1) + b + o (A / N, zero
//             outside A)
//   factors:  row-major over the shifts, [r][k][2b + 1]: l_1..l_b, ui, em_1..em_b
//             with l_i = L[r][r - i], ui = 1 / U[r][r],
//             em_j = U[r][r + j] / U[r][r] (zero outside the matrix), so the
//             backward sweep is x_r = ui z_r - sum_j em_j x_{r+j}.  One row's
//             values of all shifts are contiguous, so a block of rows is one
//             contiguous range that the wave stages through LDS
//   band_steps_kernel only:
//   vectors:  per function slot, two ping-pong buffers and one for u_1 (φ1)
//             or the hybrid set's polynomial part, d x p row-major
//   checkpoints: per slot, the last b forward values of every shift at the
//             end of each chunk of kBandL(b) rows, [chunk][k][b][p]
// A band_steps_kernel step makes two passes over the column.  The forward pass forms y = B x
// and runs the forward sweeps of all shifts, keeping only the checkpoints.
// The backward pass walks the chunks from the last: it recomputes the
// chunk's forward values from its checkpoint in registers (reading x again,
// with b rows on either side), then runs the backward sweeps of all shifts
// and forms out = a0 x + sum_k w_k x_k.  Per column-step the vector moves
// about (3 + 2b/L + 2 m b / L) d x 8 bytes instead of (3 + 2m) d x 8 when
// every forward value is stored.
#pragma once

#include "kern_common.h"
#include "kern_tri.h"

namespace pfm {

constexpr int kBandMaxB = 4;
constexpr int kBsC = 16;  // band_scan_kernel: columns per workgroup, one after another
constexpr int kBandCH = 8;  // forward pass: x rows read ahead
// rows per checkpoint chunk: the backward pass holds the chunk's forward
// values of every shift in registers (4 rows keep the kernel within the
// registers of two waves per SIMD)
__host__ __device__ constexpr int kBandL(int b) { return 4; }

struct BandDesc {
  const double *bands, *V;
  double *Fe, *Fp;
  int64_t ldv, ldf;
  int32_t d, p, b, pad_;
  double theta;
  int64_t b_off;  // B: [d][2b + 1]
  int64_t f_off;  // factors: [d][k][2b + 1]
  int64_t v_off;  // vectors: [slot][3][d][p]
  int64_t z_off;  // checkpoints: [slot][chunk][k][b][p]
  int32_t wave0;   // first wave of this instance in band_steps_kernel's launch
  int32_t nwaves;  // its waves: functions x ceil(p / 64) (0: band_scan_kernel takes it)
  int32_t sg0;     // first workgroup of this instance in band_scan_kernel's launch
  int32_t nsg;     // its workgroups: functions x ceil(p / kBsC) (0: band_steps_kernel takes it)
};

// ||A||_1 (column j adds |A[i][j]| for rows i = j - b .. j + b in increasing
// order) and N = max(1, ceil(eta / θ)); one workgroup per instance.
__global__ void __launch_bounds__(256)
band_plan_kernel(const BandDesc *__restrict__ desc, PlanRec *__restrict__ plan, int force_plan) {
  __shared__ double red[4];
  __shared__ int bad[4];
  const int ii = blockIdx.x, t = threadIdx.x;
  const BandDesc D = desc[ii];
  const int d = D.d, b = D.b;
  double mx = 0.0;
  int nan = 0;
  for (int j = t; j < d; j += 256) {
    double s = 0.0;
    for (int o = b; o >= -b; --o) {
      const int i = j - o;
      if (i >= 0 && i < d) s += fabs(D.bands[(int64_t)(b + o) * d + i]);
    }
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
  P.route = 4;
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
  // more than kNCap steps: PFM_NOT_COMPUTED, the instance is skipped
  if (P.s > kNCap) P.status |= 8;
  plan[ii] = P;
}

// B = A / N and the LU of M = I - c_k B for every (instance, shift): one
// thread each, elimination down the band without interchanges.  The rows
// q .. q + BW that elimination step q touches are held in registers (row
// r's values: l_1..l_b, then the diagonal, then U[r][r + 1..b]; they start
// as M's); step q subtracts l M[q][.] from the rows below it, normalises
// row q (1/u, em_j = U[q][q + j] / U[q][q]) and stores it, and the next row
// of M enters the window.  The instance's shifts share the writing of B.
// A zero or non-finite pivot sets PFM_SINGULAR_SHIFT with the smallest such
// shift.
template <int BW>
__global__ void __launch_bounds__(64)
band_factor_kernel(const BandDesc *__restrict__ desc, PlanRec *__restrict__ plan, int batch, TriTerms T,
                   double *__restrict__ wsd) {
  constexpr int W = 2 * BW + 1;
  const int gid = blockIdx.x * 64 + threadIdx.x;
  const int ii = gid / T.nterms, k = gid - ii * T.nterms;
  if (ii >= batch) return;
  if (plan[ii].status & 8) return;  // PFM_NOT_COMPUTED (too many steps)
  const BandDesc D = desc[ii];
  const int d = D.d, nt = T.nterms;
  const double Nd = (double)plan[ii].s;
  const double c = T.c[k];
  const double *__restrict__ A = D.bands;
  double *__restrict__ Bw = wsd + D.b_off;
  double *__restrict__ Fb = wsd + D.f_off;
  // One thread per (instance, shift) leaves the chip's SIMDs mostly empty,
  // so A's rows are loaded kFacPF at a time from clamped (in-bounds)
  // addresses, and the conditions below select on the values.
  // A's band entries at row r (clamped into the matrix), diagonal by diagonal
  auto raw_row = [&](int r, double *v) {
    const int rc = min(r, d - 1);
#pragma unroll
    for (int o = 0; o < W; ++o) v[o] = A[(int64_t)o * d + rc];
  };
  for (int r0 = k; r0 < d; r0 += kFacPF * nt) {
    double raw[kFacPF][W];
#pragma unroll
    for (int q = 0; q < kFacPF; ++q) raw_row(r0 + q * nt, raw[q]);
#pragma unroll
    for (int q = 0; q < kFacPF; ++q) {
      const int r = r0 + q * nt;
      double v[W];
#pragma unroll
      for (int o = -BW; o <= BW; ++o) v[BW + o] = (r + o >= 0 && r + o < d) ? raw[q][BW + o] / Nd : 0.0;
      if (r < d) {
#pragma unroll
        for (int o = 0; o < W; ++o) Bw[(int64_t)r * W + o] = v[o];
      }
    }
  }
  // M's row r in the window's layout (zero past the matrix) from its raw entries
  auto mrow = [&](int r, const double *a, double *v) {
#pragma unroll
    for (int i = 1; i <= BW; ++i) v[i - 1] = (r < d && r - i >= 0) ? -c * (a[BW - i] / Nd) : 0.0;
    v[BW] = r < d ? 1.0 - c * (a[BW] / Nd) : 1.0;
#pragma unroll
    for (int j = 1; j <= BW; ++j) v[BW + j] = r + j < d ? -c * (a[BW + j] / Nd) : 0.0;
  };
  double win[BW + 1][W];
#pragma unroll
  for (int r = 0; r <= BW; ++r) {
    double a[W];
    raw_row(r, a);
    mrow(r, a, win[r]);
  }
  bool bad = false;
#pragma unroll 1
  for (int q0 = 0; q0 < d; q0 += kFacPF) {
    // the rows that enter the window during this block
    double raw[kFacPF][W];
#pragma unroll
    for (int s = 0; s < kFacPF; ++s) raw_row(q0 + s + BW + 1, raw[s]);
#pragma unroll
    for (int s = 0; s < kFacPF; ++s) {
      const int q = q0 + s;
      const double piv = win[0][BW];
      bad |= q < d && !(piv != 0.0 && isfinite(piv));
#pragma unroll
      for (int i = 1; i <= BW; ++i) {
        if (q + i < d) {
          const double lv = win[i][i - 1] / piv;  // M[q + i][q] / U[q][q]
          win[i][i - 1] = lv;
#pragma unroll
          for (int j = 1; j <= BW; ++j) {
            if (q + j < d) {
              const double u = win[0][BW + j];  // U[q][q + j], not yet normalised
              const int off = j - i;            // column q + j relative to row q + i
              if (off == 0) win[i][BW] -= lv * u;
              else if (off > 0) win[i][BW + off] -= lv * u;
              else win[i][-off - 1] -= lv * u;
            }
          }
        }
      }
      const double inv = 1.0 / piv;
      win[0][BW] = inv;
#pragma unroll
      for (int j = 1; j <= BW; ++j) win[0][BW + j] *= inv;
      if (q < d) {
        double *out = Fb + ((int64_t)q * nt + k) * W;
#pragma unroll
        for (int j = 0; j < W; ++j) out[j] = win[0][j];
      }
#pragma unroll
      for (int r = 0; r < BW; ++r)
#pragma unroll
        for (int j = 0; j < W; ++j) win[r][j] = win[r + 1][j];
      mrow(q + BW + 1, raw[s], win[BW]);
    }
  }
  if (bad) {
    atomicOr(&plan[ii].status, 1);
    atomicMin(&plan[ii].bad_shift, k);
  }
}

// All N steps of one column (lane) of one function slot; 64 consecutive
// columns of one instance per wave.  BW is the half-bandwidth b.  The
// forward pass keeps windows of x (2 BW + 1 rows, y_r = sum_o B[r][r+o]
// x_{r+o} needs x_{r+BW}) and, for the hybrid set, of y (P_s =
// d1 y_s + d2 (B y)_s needs y_{s+BW}); the sweeps keep the last BW values of
// every shift.  NT is the number of shifts (4, 5, 8 or 10), so the
// windows are sized to the set and stay in registers.  B and the factor rows
// of each block (kBandCH rows forward, kBandL rows backward) are loaded by
// all 64 lanes with vector loads one block ahead, written to the LDS buffer
// not being read, and read by the sweeps as broadcasts; the workgroup is one
// wave, so its barriers only order the LDS accesses.  Lanes past p follow
// column p - 1 and store nothing: apart from the staged rows, every value a
// lane uses was written by a lane of its own column.  For b <= 2 the kernel
// is held to the registers of two waves per SIMD: it spills about 150 bytes
// per lane (b = 2, m = 8) and still runs 1.4x faster than one wave without
// spills; wider bands spill far more and keep one wave.
template <int BW, int NT>
__global__ void __launch_bounds__(64, BW <= 2 ? 2 : 1)
band_steps_kernel(const BandDesc *__restrict__ desc, int batch, const PlanRec *__restrict__ plan, TriTerms T,
                  const double *__restrict__ fac, double *__restrict__ vws) {
  const int lane = threadIdx.x;
  const int gw = blockIdx.x;
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].wave0 <= gw) lo = mid;
    else hi = mid - 1;
  }
  if (plan[lo].status & 8) return;  // PFM_NOT_COMPUTED: the whole wave leaves before any barrier
  const BandDesc D = desc[lo];
  const int d = D.d, p = D.p;
  const int ncw = (p + 63) / 64;
  const int w = gw - D.wave0;
  const int slot = w / ncw;
  // lanes past p follow column p - 1 and store nothing (every lane takes
  // part in staging the factor rows)
  const bool active = (w - slot * ncw) * 64 + lane < p;
  const int c = active ? (w - slot * ncw) * 64 + lane : p - 1;
  const int fn = T.fn[slot];
  constexpr int nt = NT;
  const int N = plan[lo].s;
  const bool hyb = T.d1 != 0.0 || T.d2 != 0.0;
  const int64_t dp = (int64_t)d * p;
  const double *Bw = fac + D.b_off;
  const double *F0 = fac + D.f_off;
  constexpr int W = 2 * BW + 1;                     // values per row and shift
  double *buf0 = vws + D.v_off + (int64_t)slot * 3 * dp, *buf1 = buf0 + dp, *ub = buf1 + dp;
  constexpr int LC = kBandL(BW);
  const int nch = (d + LC - 1) / LC;
  const int64_t ckst = (int64_t)nt * BW * p;  // one chunk's checkpoints
  double *ckb = vws + D.z_off + (int64_t)slot * nch * ckst;
  double *out_final = fn ? D.Fp : D.Fe;
  // factor rows staged through LDS: row u of a block holds B's row, then the
  // W values of every shift (R doubles); blocks of SB rows, two buffers
  constexpr int R = (NT + 1) * W;
  constexpr int SF = kBandCH, SBK = LC;               // rows per block: forward, backward
  constexpr int PL = (SF * R + 63) / 64;              // values per lane per forward block
  __shared__ double st[2][SF * R];
  double sv[PL];
  // this lane's share of the block of n rows from row r0 (rows past d as 0)
  auto stage_load = [&](int r0, int n) {
#pragma unroll
    for (int i = 0; i < PL; ++i) {
      const int e = lane + 64 * i;
      const int u = e / R, q = e - u * R;
      const int r = r0 + u;
      double v = 0.0;
      if (e < n * R && r >= 0 && r < d)
        v = q < W ? gld(Bw + (int64_t)r * W + q) : gld(F0 + (int64_t)r * NT * W + (q - W));
      sv[i] = v;
    }
  };
  auto stage_put = [&](int buf, int n) {
#pragma unroll
    for (int i = 0; i < PL; ++i) {
      const int e = lane + 64 * i;
      if (e < n * R) st[buf][e] = sv[i];
    }
  };

  for (int j = 0; j < N; ++j) {
    const double *src = j == 0 ? D.V : ((j - 1) & 1 ? buf1 : buf0);
    const int64_t lds = j == 0 ? D.ldv : p;
    double *dst = j == N - 1 ? out_final : (j & 1 ? buf1 : buf0);
    const int64_t ldd = j == N - 1 ? D.ldf : p;
    const bool first_phi = fn == 1 && j == 0;
    const bool add = (fn == 1 && j > 0) || hyb;
    const bool keep_u1 = first_phi && N > 1;
    // φ1's first step is rho(B) V / N: the 1/N goes into its weights
    const double a0 = first_phi ? T.a0p / N : T.a0e;
    double wts[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) wts[k] = first_phi ? T.wp[k] / N : T.we[k];

    // forward pass over blocks of SF rows: x read one block ahead, the
    // block's factor rows from LDS (staged while the previous block ran)
    {
      double xw[2 * BW + 1], yw[2 * BW + 1], zw[NT][BW], xn[SF];
#pragma unroll
      for (int q = 0; q <= 2 * BW; ++q) xw[q] = yw[q] = 0.0;
#pragma unroll
      for (int k = 0; k < NT; ++k)
#pragma unroll
        for (int i = 0; i < BW; ++i) zw[k][i] = 0.0;
      // rows r < rend are visited: y and z for r < d, the hybrid set's P
      // one window behind (rows past d have y = 0)
      const int rend = d + (hyb ? BW : 0);
      const int nbl = (rend + SF - 1) / SF;
      // x_0 .. x_{BW-1} enter the window first; block i then pushes
      // x_{r0 + BW} .. x_{r0 + SF - 1 + BW}
#pragma unroll
      for (int t = 0; t < BW; ++t) {
#pragma unroll
        for (int q = 0; q < 2 * BW; ++q) xw[q] = xw[q + 1];
        xw[2 * BW] = t < d ? gld(src + (int64_t)t * lds + c) : 0.0;
      }
      auto load_x = [&](int r0) {
#pragma unroll
        for (int u = 0; u < SF; ++u) {
          const int t = r0 + BW + u;
          xn[u] = t < d ? gld(src + (int64_t)t * lds + c) : 0.0;
        }
      };
      load_x(0);
      stage_load(0, SF);
      __syncthreads();  // the previous step's last chunk has read its buffer
      stage_put(0, SF);
      __syncthreads();
      for (int bi = 0; bi < nbl; ++bi) {
        const int r0 = bi * SF;
        const double *sb = st[bi & 1];
        double xc[SF];
#pragma unroll
        for (int u = 0; u < SF; ++u) xc[u] = xn[u];
        if (bi + 1 < nbl) {
          load_x(r0 + SF);
          stage_load(r0 + SF, SF);
        }
#pragma unroll
        for (int u = 0; u < SF; ++u) {
          const int r = r0 + u;
          if (r < rend) {
#pragma unroll
            for (int q = 0; q < 2 * BW; ++q) xw[q] = xw[q + 1];
            xw[2 * BW] = xc[u];
            const double *fr = sb + u * R;
            double y = 0.0;
            if (r < d) {
#pragma unroll
              for (int o = -BW; o <= BW; ++o) y = fma(fr[BW + o], xw[BW + o], y);
#pragma unroll
              for (int k = 0; k < NT; ++k) {
                double z = y;
#pragma unroll
                for (int i = 1; i <= BW; ++i) z = fma(-fr[W + k * W + i - 1], zw[k][BW - i], z);
#pragma unroll
                for (int i = 0; i + 1 < BW; ++i) zw[k][i] = zw[k][i + 1];
                zw[k][BW - 1] = z;
              }
              // checkpoint for the chunk that starts at row r + 1
              if ((r + 1) % LC == 0 && r + 1 < d && active) {
                double *cq = ckb + (int64_t)((r + 1) / LC) * ckst + c;
#pragma unroll
                for (int k = 0; k < NT; ++k)
#pragma unroll
                  for (int i = 0; i < BW; ++i) cq[(int64_t)(k * BW + i) * p] = zw[k][i];
              }
            }
            if (hyb) {
#pragma unroll
              for (int q = 0; q < 2 * BW; ++q) yw[q] = yw[q + 1];
              yw[2 * BW] = y;
              const int s = r - BW;
              if (s >= 0 && s < d) {
                double by = 0.0;
#pragma unroll
                for (int o = -BW; o <= BW; ++o) by = fma(Bw[(int64_t)s * W + BW + o], yw[BW + o], by);
                if (active) ub[(int64_t)s * p + c] = fma(T.d2, by, T.d1 * yw[BW]);
              }
            }
          }
        }
        if (bi + 1 < nbl) {
          __syncthreads();  // every lane is done with the other buffer
          stage_put((bi + 1) & 1, SF);
          __syncthreads();
        }
      }
    }

    // backward pass, chunk by chunk from the last
    {
      double xk[NT][BW];  // xk[k][i] = x_{k, r + 1 + i}
#pragma unroll
      for (int k = 0; k < NT; ++k)
#pragma unroll
        for (int i = 0; i < BW; ++i) xk[k][i] = 0.0;
      __syncthreads();
      stage_load((nch - 1) * LC, SBK);
      stage_put(0, SBK);
      __syncthreads();
      for (int q = nch - 1; q >= 0; --q) {
        const int r0 = q * LC;
        const double *sb = st[(nch - 1 - q) & 1];
        if (q > 0) stage_load(r0 - LC, SBK);
        // x_{r0 - BW} .. x_{r0 + LC - 1 + BW} (zero outside the vector), u_1
        // or P, and the checkpoint z_{k, r0 - BW} .. z_{k, r0 - 1}
        double xh[LC + 2 * BW], us[LC], zc[NT][LC], zk[NT][BW];
#pragma unroll
        for (int i = 0; i < LC + 2 * BW; ++i) {
          const int r = r0 - BW + i;
          xh[i] = (r >= 0 && r < d) ? gld(src + (int64_t)r * lds + c) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LC; ++u) us[u] = (add && r0 + u < d) ? gld(ub + (int64_t)(r0 + u) * p + c) : 0.0;
        {
          const double *cq = ckb + (int64_t)q * ckst + c;
#pragma unroll
          for (int k = 0; k < NT; ++k)
            if (k < nt)
#pragma unroll
              for (int i = 0; i < BW; ++i) zk[k][i] = q > 0 ? gld(cq + (int64_t)(k * BW + i) * p) : 0.0;
        }
        // the chunk's forward values, in registers
#pragma unroll
        for (int u = 0; u < LC; ++u) {
          const int r = r0 + u;
          if (r < d) {
            double y = 0.0;
#pragma unroll
            for (int o = -BW; o <= BW; ++o) y = fma(sb[u * R + BW + o], xh[BW + u + o], y);
#pragma unroll
            for (int k = 0; k < NT; ++k) {
              if (k < nt) {
                const double *Fk = sb + u * R + W + k * W;
                double z = y;
#pragma unroll
                for (int i = 1; i <= BW; ++i) {
                  const double zp = u - i >= 0 ? zc[k][u - i >= 0 ? u - i : 0] : zk[k][BW + u - i >= 0 ? BW + u - i : 0];
                  z = fma(-Fk[i - 1], zp, z);
                }
                zc[k][u] = z;
              }
            }
          }
        }
        // the backward sweeps and the combination
#pragma unroll
        for (int u = LC - 1; u >= 0; --u) {
          const int r = r0 + u;
          if (r < d) {
            double o = fma(a0, xh[BW + u], us[u]);
#pragma unroll
            for (int k = 0; k < NT; ++k) {
              if (k < nt) {
                const double *Fk = sb + u * R + W + k * W;
                double x = Fk[BW] * zc[k][u];
#pragma unroll
                for (int jj = 1; jj <= BW; ++jj) x = fma(-Fk[BW + jj], xk[k][jj - 1], x);
#pragma unroll
                for (int i = BW - 1; i > 0; --i) xk[k][i] = xk[k][i - 1];
                xk[k][0] = x;
                o = fma(wts[k], x, o);
              }
            }
            if (active) {
              dst[(int64_t)r * ldd + c] = o;
              if (keep_u1) ub[(int64_t)r * p + c] = o;
            }
          }
        }
        if (q > 0) {
          __syncthreads();
          stage_put((nch - q) & 1, SBK);
          __syncthreads();
        }
      }
    }
  }
}

// All N steps of the pentadiagonal action (b = 2, d <= kTsMaxD, up to 8
// shifts), one column at a time per workgroup and a wave per shift.  Lane L
// of wave k holds rows 16 L .. 16 L + 15 of shift k's factors (l_1, l_2,
// 1/u, em_1, em_2) in registers for the whole launch; B, the column's y and
// B y, and the shifts' w_k x_k live in LDS, transposed so that the lanes'
// accesses to one row index are consecutive (row r at (r % 16) 64 + r / 16).
// A step:
//   f = B y                 (the workgroup, a thread per pair of adjacent rows)
//   forward  z_r = f_r - l_1 z_{r-1} - l_2 z_{r-2}: each lane's 16 rows from
//            a zero state give the state leaving them, h_L = (z_{14}, z_{15});
//            with the lane's homogeneous 2 x 2 map M_L (formed once) the state
//            entering lane L is h_{L-1} + M_{L-1} h_{L-2} when every map entry
//            is at most 2^-30 (the rest, M_{L-1} M_{L-2} h_{L-3}, is below
//            2^-58 of the largest state; lane L - 1 forms it with its own map
//            and DPP moves it up), else the maps are composed lane by lane;
//            the lane then sweeps its rows again from that state
//   backward x_r = ui_r z_r - em_1 x_{r+1} - em_2 x_{r+2}: the same from lane
//            63 down, and w_k x_k into LDS (exp alone: w_k ui is held in place
//            of ui, so the sweep gives w_k x_k itself)
//   y <- a0 y (+ u_1) + sum_k w_k x_k   (the workgroup, by rows, k in order)
// Three barriers per step; the columns of a workgroup run one after another,
// so the factors are loaded once for kBsC columns.
template <int NT, bool PHI>
__global__ void __launch_bounds__(64 * NT)
band_scan_kernel(const BandDesc *__restrict__ desc, int batch, const PlanRec *__restrict__ plan, TriTerms T,
                 const double *__restrict__ fac, int nsg) {
  constexpr int R = 16, NTH = 64 * NT, MD = kTsMaxD;
  __shared__ double Bs[5 * MD];   // B[r][r + o] at (o + 2) MD + (r % 16) 64 + r / 16
  __shared__ double ys[16 * 65];  // y: row r at (r % 16) 65 + r / 16 + 1; column 0 is zero
  __shared__ double fs[MD];       // B y
  __shared__ double part[NT * MD];  // w_k x_k
  __shared__ double maps[NT * 64 * 8];  // per (shift, lane): M (row-major), then G
  const int t = threadIdx.x, lane = t & 63, k = t >> 6;
  // workgroup b runs on XCD b mod 8: XCD x takes the x-th eighth of the
  // workgroups in order, so the workgroups of one instance share an L2
  const int sgw = (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3));
  if (sgw >= nsg) return;  // grid padding: uniform, before any barrier
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].sg0 <= sgw) lo = mid;
    else hi = mid - 1;
  }
  const int ii = lo;
  if (plan[ii].status & 8) return;  // PFM_NOT_COMPUTED: uniform, before any barrier
  const BandDesc D = desc[ii];
  const int d = D.d, p = D.p;
  const int cpg = (p + kBsC - 1) / kBsC;
  const int wl = sgw - D.sg0;
  const int slot = wl / cpg;
  const int c0 = (wl - slot * cpg) * kBsC;
  const int fn = slot == 0 ? T.fn[0] : T.fn[1];
  const int N = plan[ii].s;
  const double *Bw = fac + D.b_off;  // [r][5]
  const double *Fw = fac + D.f_off;  // [r][k][5]

  if (t < 16) ys[t * 65] = 0.0;  // the zero column, never written again
  // B into LDS: a thread per (diagonal, lane), its 16 rows
  for (int q = t; q < 5 * 64; q += NTH) {
    const int o = q >> 6, L = q & 63;
    double v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = L * R + i;
      v[i] = r < d ? Bw[(int64_t)r * 5 + o] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) Bs[o * MD + i * 64 + L] = v[i];
  }
  // this wave's shift, this lane's rows
  double l1[R], l2[R], ui[R], e1[R], e2[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = lane * R + i;
    const double *f = Fw + ((int64_t)r * NT + k) * 5;
    const bool in = r < d;
    l1[i] = in ? f[0] : 0.0;
    l2[i] = in ? f[1] : 0.0;
    ui[i] = in ? f[2] : 0.0;
    e1[i] = in ? f[3] : 0.0;
    e2[i] = in ? f[4] : 0.0;
  }
  // exp alone: w_k is the same at every step, and w_k x obeys the backward
  // recurrence with w_k ui in place of ui, so the weight is folded in here
  if constexpr (!PHI) {
    const double w = T.we[k];
#pragma unroll
    for (int i = 0; i < R; ++i) ui[i] *= w;
  }
  // the lane's homogeneous maps: forward (z_{-2}, z_{-1}) -> (z_14, z_15),
  // backward (x_16, x_17) -> (x_0, x_1), column by column
  double M[2][2], G[2][2];
#pragma unroll
  for (int cidx = 0; cidx < 2; ++cidx) {
    double zm2 = cidx == 0 ? 1.0 : 0.0, zm1 = cidx == 0 ? 0.0 : 1.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const double z = fma(-l1[i], zm1, -l2[i] * zm2);
      zm2 = zm1;
      zm1 = z;
    }
    M[0][cidx] = zm2;
    M[1][cidx] = zm1;
    double xp1 = cidx == 0 ? 1.0 : 0.0, xp2 = cidx == 0 ? 0.0 : 1.0;
#pragma unroll
    for (int i = R - 1; i >= 0; --i) {
      const double x = fma(-e1[i], xp1, -e2[i] * xp2);
      xp2 = xp1;
      xp1 = x;
    }
    G[0][cidx] = xp1;
    G[1][cidx] = xp2;
  }
  const double thr = 0x1p-30;
  const bool short_scan = !__any(!(fabs(M[0][0]) <= thr && fabs(M[0][1]) <= thr && fabs(M[1][0]) <= thr &&
                                   fabs(M[1][1]) <= thr && fabs(G[0][0]) <= thr && fabs(G[0][1]) <= thr &&
                                   fabs(G[1][0]) <= thr && fabs(G[1][1]) <= thr));
  {
    double *mp = maps + (k * 64 + lane) * 8;
    mp[0] = M[0][0]; mp[1] = M[0][1]; mp[2] = M[1][0]; mp[3] = M[1][1];
    mp[4] = G[0][0]; mp[5] = G[0][1]; mp[6] = G[1][0]; mp[7] = G[1][1];
  }
  const double *mk = maps + k * 64 * 8;  // this wave's maps, lane by lane
  __syncthreads();

  constexpr int NQ = (16 + NT - 1) / NT;  // row indices i per thread in the by-rows phases
#pragma unroll 1
  for (int cc = 0; cc < kBsC; ++cc) {
    const int col = c0 + cc;
    if (col >= p) break;  // uniform over the workgroup
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = q * NT + k;
      if (i < 16) {
        const int r = lane * R + i;
        ys[i * 65 + lane + 1] = r < d ? D.V[(int64_t)r * D.ldv + col] : 0.0;
      }
    }
    double u1[PHI ? NQ : 1];
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
      // phi1's first step is u_1 = rho(B) V / N: the 1/N is folded into its weights
      const bool first_phi = PHI && fn == 1 && j == 0;
      const double a0 = first_phi ? T.a0p / (double)N : T.a0e;
      const double wk = first_phi ? T.wp[k] / (double)N : T.we[k];
      // f = B y: a thread takes NQ adjacent rows of its lane's block, so
      // their y values are read once, NQ + 4 of them
      {
        const int i0 = k * NQ;
        if (i0 < 16) {
          double yw[NQ + 4];
#pragma unroll
          for (int q = 0; q < NQ + 4; ++q) {
            const int rr = lane * R + i0 + q - 2;
            yw[q] = ys[(rr & 15) * 65 + (rr >> 4) + 1];  // rows -2, -1, MD, MD + 1: column 0
          }
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const int i = i0 + q;
            if (i < 16) {
              double f = 0.0;
#pragma unroll
              for (int o = -2; o <= 2; ++o) f = fma(Bs[(o + 2) * MD + i * 64 + lane], yw[q + o + 2], f);
              fs[i * 64 + lane] = f;
            }
          }
        }
      }
      __syncthreads();
      // forward: the state leaving this lane's rows from a zero state (its
      // first two rows need no terms of the state)
      double fr[R];
      fr[0] = fs[lane];
      fr[1] = fs[64 + lane];
      double zm2 = fr[0], zm1 = fma(-l1[1], fr[0], fr[1]);
#pragma unroll
      for (int i = 2; i < R; ++i) {
        fr[i] = fs[i * 64 + lane];
        const double z = fma(-l1[i], zm1, fma(-l2[i], zm2, fr[i]));
        zm2 = zm1;
        zm1 = z;
      }
      double s0, s1;  // the state entering this lane: (z_{-2}, z_{-1})
      if (short_scan) {
        const double h10 = dpp0_f64<0x138>(zm2), h11 = dpp0_f64<0x138>(zm1);  // wave_shr:1
        if constexpr (!PHI) {
          // lane L forms h_L + M_L h_{L-1} with its own map (registers); one
          // shift up gives lane L + 1 its entering state
          const double c0 = fma(M[0][0], h10, fma(M[0][1], h11, zm2));
          const double c1 = fma(M[1][0], h10, fma(M[1][1], h11, zm1));
          s0 = dpp0_f64<0x138>(c0);
          s1 = dpp0_f64<0x138>(c1);
        } else {
          // phi1 keeps u_1 too: the neighbour's map from LDS, so nothing spills
          const double h20 = dpp0_f64<0x138>(h10), h21 = dpp0_f64<0x138>(h11);
          const double *m = mk + (lane > 0 ? lane - 1 : 0) * 8;  // M_{L-1} (lane 0: h1 = h2 = 0)
          s0 = fma(m[0], h20, fma(m[1], h21, h10));
          s1 = fma(m[2], h20, fma(m[3], h21, h11));
        }
      } else {
        double a0s = 0.0, a1s = 0.0;
        s0 = 0.0;
        s1 = 0.0;
        for (int L = 0; L < 64; ++L) {
          if (lane == L) {
            s0 = a0s;
            s1 = a1s;
          }
          const double *m = mk + L * 8;
          const double n0 = fma(m[0], a0s, fma(m[1], a1s, readlane_f64(zm2, L)));
          const double n1 = fma(m[2], a0s, fma(m[3], a1s, readlane_f64(zm1, L)));
          a0s = n0;
          a1s = n1;
        }
      }
      // the rows again from the entering state; keep ui z
      double sv[R];
      zm2 = s0;
      zm1 = s1;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const double z = fma(-l1[i], zm1, fma(-l2[i], zm2, fr[i]));
        zm2 = zm1;
        zm1 = z;
        sv[i] = ui[i] * z;
      }
      // backward: the state leaving this lane upwards from a zero state
      double xp2 = sv[R - 1], xp1 = fma(-e1[R - 2], sv[R - 1], sv[R - 2]);
#pragma unroll
      for (int i = R - 3; i >= 0; --i) {
        const double x = fma(-e1[i], xp1, fma(-e2[i], xp2, sv[i]));
        xp2 = xp1;
        xp1 = x;
      }
      double x0, x1;  // the state entering this lane from below: (x_16, x_17)
      if (short_scan) {
        const double h10 = dpp0_f64<0x130>(xp1), h11 = dpp0_f64<0x130>(xp2);  // wave_shl:1
        if constexpr (!PHI) {
          const double c0 = fma(G[0][0], h10, fma(G[0][1], h11, xp1));
          const double c1 = fma(G[1][0], h10, fma(G[1][1], h11, xp2));
          x0 = dpp0_f64<0x130>(c0);
          x1 = dpp0_f64<0x130>(c1);
        } else {
          const double h20 = dpp0_f64<0x130>(h10), h21 = dpp0_f64<0x130>(h11);
          const double *g = mk + (lane < 63 ? lane + 1 : 63) * 8 + 4;  // G_{L+1} (lane 63: h1 = h2 = 0)
          x0 = fma(g[0], h20, fma(g[1], h21, h10));
          x1 = fma(g[2], h20, fma(g[3], h21, h11));
        }
      } else {
        double a0s = 0.0, a1s = 0.0;
        x0 = 0.0;
        x1 = 0.0;
        for (int L = 63; L >= 0; --L) {
          if (lane == L) {
            x0 = a0s;
            x1 = a1s;
          }
          const double *g = mk + L * 8 + 4;
          const double n0 = fma(g[0], a0s, fma(g[1], a1s, readlane_f64(xp1, L)));
          const double n1 = fma(g[2], a0s, fma(g[3], a1s, readlane_f64(xp2, L)));
          a0s = n0;
          a1s = n1;
        }
      }
      xp1 = x0;
      xp2 = x1;
#pragma unroll
      for (int i = R - 1; i >= 0; --i) {
        const double x = fma(-e1[i], xp1, fma(-e2[i], xp2, sv[i]));
        xp2 = xp1;
        xp1 = x;
        part[k * MD + i * 64 + lane] = PHI ? wk * x : x;
      }
      __syncthreads();
      // y <- a0 y (+ u_1) + sum_k w_k x_k
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = q * NT + k;
        if (i < 16) {
          const int e = i * 64 + lane;
          double a = a0 * ys[e + i + 1];
          if constexpr (PHI) {
            if (fn == 1 && j > 0) a += u1[q];
          }
#pragma unroll
          for (int kk = 0; kk < NT; ++kk) a += part[kk * MD + e];
          if constexpr (PHI) {
            if (first_phi && N > 1) u1[q] = a;
          }
          ys[e + i + 1] = a;
        }
      }
      __syncthreads();
    }
    double *F = (fn ? D.Fp : D.Fe) + col;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = q * NT + k;
      if (i < 16) {
        const int r = lane * R + i;
        if (r < d) F[(int64_t)r * D.ldf] = ys[i * 65 + lane + 1];
      }
    }
    __syncthreads();  // the next column overwrites ys
  }
}

__global__ void __launch_bounds__(256)
band_info_kernel(const BandDesc *__restrict__ desc, const PlanRec *__restrict__ plan, InfoRec *__restrict__ info,
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
