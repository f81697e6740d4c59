// Common device helpers for the gfx950 kernels of libpfm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfm_internal.h"

namespace pfm {

typedef double v4d __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64: D(16x16) = A(16x4) * B(4x16) + C.
// Hardware fragment layout (checked on the device by pfm_selftest_mfma):
// lane l = 16 g + i (i = l & 15, g = l >> 4) supplies A[i][g] and B[g][i] and
// holds D[g + 4 v][i] in element v of the accumulator.
//
// The kernels feed the A operand with its rows permuted by
// arow(i) = 4 (i & 3) + (i >> 2); then element v of lane (g, i) holds the
// product's row 4 g + v, so each lane owns four *contiguous* rows of a
// column and tiles load and store as 32-byte vectors.  Every A fragment below
// is therefore read at row arow(i16), and every C fragment is read or
// written at rows 4 g + v.
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int arow(int i16) { return ((i16 & 3) << 2) | (i16 >> 2); }

__device__ __forceinline__ v4d zero4() {
  v4d z = {0.0, 0.0, 0.0, 0.0};
  return z;
}

typedef float v4f __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x4_f32 (binary32 path).  Operand layout as above; element v
// of lane (g, i) holds D[4 g + v][i] (checked by pfm_selftest_mfma32), so the
// A operand is fed unpermuted.
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Element-type traits shared by the templated LU and substitution kernels.
template <class S> struct MT;
template <> struct MT<double> {
  typedef v4d v4;
  static __device__ __forceinline__ int arow_(int i16) { return arow(i16); }
  static __device__ __forceinline__ v4 zero() { return zero4(); }
};
template <> struct MT<float> {
  typedef v4f v4;
  static __device__ __forceinline__ int arow_(int i16) { return i16; }
  static __device__ __forceinline__ v4 zero() { v4f z = {0.f, 0.f, 0.f, 0.f}; return z; }
};

// Order LDS traffic of one wave (write then read by other lanes of it).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup -> (instance slot, sub-task) mapping that keeps every sub-task of
// one instance on the same XCD (workgroups are dealt round-robin to the 8
// XCDs), so the instance's data is shared through one L2.
__device__ __forceinline__ void xcd_map(int bid, int nsub, int &slot, int &sub) {
  const int x = bid & 7, q = bid >> 3;
  sub = q % nsub;
  slot = (q / nsub) * 8 + x;
}

__host__ __device__ __forceinline__ int xcd_grid(int nslots, int nsub) {
  return ((nslots + 7) / 8) * 8 * nsub;
}

}  // namespace pfm
