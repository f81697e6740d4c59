// Internal structures shared by the host runtime and the kernels of libpfm.
#pragma once
#include <stdint.h>

namespace pfm {

constexpr int kMaxTerms = 16;   // nonzero-shift solves per call
constexpr int kSCap = 1000;     // largest squaring count accepted
constexpr int kNCap = 1 << 20;  // largest action step count accepted
constexpr int kSqTile = 64;     // squaring GEMM tile edge

// One problem instance as the kernels see it.  Offsets index the context's
// workspace (doubles for *_off in the double region, ints for *_ioff).
struct InstDesc {
  const double *A;   // caller's A (row-major; complex: interleaved)
  const double *V;   // caller's V (action), else null
  double *Fe;        // caller's outputs (row-major)
  double *Fp;
  int64_t lda, ldv, ldf;
  int32_t n, npad, p, cls;
  int64_t fac_off;   // nterms * npad^2 (complex: 2x) : LU factors, column-major
  int64_t dinv_off;  // nterms * 2 * (npad/16) * 256   : inverted 16x16 diagonal blocks of L and U
  int64_t r_off;     // 4 * npad^2 : R ping-pong buffers, then phi1 ping-pong buffers
  int64_t x_off;     // action: npad * p-sized state vectors
  int64_t perm_ioff; // nterms * npad : row permutation of each factorisation
  int64_t ipiv_ioff; // nterms * npad : LAPACK-style pivot sequence
};

// Device-side plan of one instance.
struct PlanRec {
  int32_t s;          // squarings (full) or N steps (action)
  int32_t status;     // PFM_* status bits
  int32_t bad_shift;  // smallest shift index with a zero pivot (0x7fffffff: none)
  int32_t ir_iters;
  double eta;         // ||A||_1
  double resid;
};

// The shift/weight list of a call (passed by value to kernels).
struct Terms {
  int32_t nterms;
  int32_t pair;        // 1: real A with complex-conjugate pairs -> combine 2 Re(w Z)
  int32_t want_exp, want_phi;
  double a0e, a0p;
  double c_re[kMaxTerms], c_im[kMaxTerms];
  double we_re[kMaxTerms], we_im[kMaxTerms];
  double wp_re[kMaxTerms], wp_im[kMaxTerms];
};

}  // namespace pfm
