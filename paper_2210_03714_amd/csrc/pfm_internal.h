// Internal structures shared by the host runtime and the kernels of libpfm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfm {

constexpr int kMaxTerms = 16;   // nonzero-shift solves per call
constexpr int kSCap = 1000;     // largest squaring count accepted
constexpr int kNCap = 1 << 20;  // largest action step count accepted
constexpr int kSqTile = 64;     // squaring GEMM tile edge
constexpr int kLargeMax = 16384; // largest real dimension (2n for complex) of a large instance
constexpr int kLnMin = 128;      // action / complex instances above this may take the multi-workgroup route

// One problem instance as the kernels see it.  Offsets index the context's
// workspace (doubles for *_off in the double region, ints for *_ioff).
//
// Complex problems run on the real embedding of a complex matrix,
// emb(X + iY) = [[X, -Y], [Y, X]] (size 2n): emb(f(A)) = f(emb(A)) for the
// real-coefficient functions here, and a complex scalar c acts as
// c_re I + c_im J with J = emb(i I).  For such instances (emb = 1) A points at
// the embedded matrix built in the workspace, n = 2 hn, and only the first
// block column (hn columns) of every n x n result is computed.
struct InstDesc {
  const double *A;   // row-major real matrix the kernels read (embedded if emb)
  const double *Ain; // caller's A (the norm is taken on it; complex: interleaved)
  const double *V;   // caller's V (action), else null
  double *Fe;        // caller's outputs (row-major): exp, phi1, phi2
  double *Fp;
  double *Fq;
  int64_t lda, ldv, ldf;
  int64_t ldin;      // leading dimension of Ain
  int32_t n, npad, p, cls;
  int32_t emb;       // 1: complex embedding, A is 2 hn x 2 hn
  int32_t hn;        // emb: size of the original problem
  int32_t cin;       // 1: caller's data are complex (interleaved)
  int32_t ncol;      // columns of the result that are computed (n, or hn if emb)
  int64_t fac_off;   // nterms * npad^2 (complex: 2x) : LU factors, column-major
  int64_t dinv_off;  // nterms * 2 * (npad/16) * 256   : inverted 16x16 diagonal blocks of L and U
  int64_t r_off;     // 4 (6 with phi2) * npad^2 : R, phi1 (and phi2) ping-pong buffers
  int64_t e_off;     // emb: the embedded matrix, row-major n x n
  double theta;      // admissible ||B||_1 for this instance's tolerance (§3)
  int64_t ln_off;    // large instances: nterms * ln_stride(npad) (colbuf, dinv)
  int64_t v_off;     // large action instances: step vectors and partial products
  int64_t perm_ioff; // nterms * npad : row permutation of each factorisation
  int64_t ipiv_ioff; // nterms * npad : LAPACK-style pivot sequence
  int32_t rflags;    // kRf* bits: the routes this instance may take (from its size alone)
  int32_t rpad_;
};

// Routes an instance may take, fixed by the host from the sizes; the device
// picks among them after the plan (route_kernel).
constexpr int kRfMayLn = 1;  // the multi-workgroup Gauss-Jordan route (action / complex above the threshold)
constexpr int kRfLarge = 2;  // n > 512: that route only
constexpr int kRfGj = 4;     // the single-workgroup Gauss-Jordan route (real full matrices)

// Device-side plan of one instance.
struct PlanRec {
  int32_t s;          // squarings (full) or N steps (action)
  int32_t status;     // PFM_* status bits
  int32_t bad_shift;  // smallest shift index with a zero pivot (0x7fffffff: none)
  int32_t ir_iters;
  int32_t route;      // 0: pivoting LU route, 1: Gauss-Jordan inverses, 2: the multi-workgroup route
  int32_t pad_;
  double eta;         // ||A||_1
  double resid;
};

// The instance takes route r and is computed (kernels of every route are
// launched over all candidates; the others return at once).
__host__ __device__ inline bool on_route(const PlanRec &P, int r) { return P.route == r && !(P.status & 8); }

// The shift/weight list of a call (passed by value to kernels).
// Real weights (fold = 0): Z_k is accumulated as we_k Z_k and wp_k Z_k.
// Complex weight (fold = 1, embedded instances): the weight of function fn_k
// is folded into the right-hand side, M_k^{-1} emb(w_k B), since M_k^{-1}
// commutes with J; the solve returns emb(w_k Z_k) directly.
// pair_real: the set is one conjugate pair per function on a real A, so the
// pair contributes 2 Re(w_k Z_k) = twice the top half of emb(w_k Z_k).
struct Terms {
  int32_t nterms;
  int32_t pair_real;
  int32_t want_exp, want_phi;  // want_phi: the phi1 chain is computed (also for phi2)
  int32_t want_phi2, pad_;
  double a0e, a0p, a0q;         // a0q, wq_re: phi2 (real shift sets, no folding)
  double d1e, d2e;  // polynomial part d1 B + d2 B^2 of the hybrid set (exp), else 0
  double c_re[kMaxTerms], c_im[kMaxTerms];
  double we_re[kMaxTerms], we_im[kMaxTerms];
  double wp_re[kMaxTerms], wp_im[kMaxTerms];
  double wq_re[kMaxTerms];
  int32_t fold[kMaxTerms];
  int32_t fn[kMaxTerms];
};

}  // namespace pfm
