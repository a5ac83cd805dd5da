// Register-blocked FIR of the pulse (Eq. axial_sig) over an LDS copy of its
// input: each thread forms kPulseR consecutive outputs and slides a window of
// 2 kPulseR inputs over the taps, so that one LDS read feeds kPulseR
// multiply-adds (the filter is bound by fp32 FMA issue, not by LDS).
#pragma once

#include <hip/hip_runtime.h>

namespace usrt {

constexpr int kPulseR = 8;
constexpr int kMaxTaps = 512;

// Padded tap count: the 2M + 1 taps rounded up to a multiple of kPulseR.
__host__ __device__ __forceinline__ int fir_padded(int M) { return (2 * M + 1 + kPulseR - 1) / kPulseR * kPulseR; }

// out[r] = sum_{q < Tp} x[b + r + q] c[q], r < R (x holds the input from M
// samples before the first output; c the reversed taps, zero past 2M + 1).
// The taps are taken kPulseR at a time; every output sums its products in
// the order q = 0, 1, .., Tp - 1 whatever R is, so the outputs do not depend
// on R (R a multiple of kPulseR).
template <int R = kPulseR>
__device__ __forceinline__ void fir_block(const float* x, const float* c, int b, int Tp, float out[R]) {
  float v[R + kPulseR];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    out[r] = 0.0f;
    v[r] = x[b + r];
  }
  for (int q0 = 0; q0 < Tp; q0 += kPulseR) {
#pragma unroll
    for (int r = 0; r < kPulseR; ++r) v[R + r] = x[b + q0 + R + r];
#pragma unroll
    for (int qq = 0; qq < kPulseR; ++qq) {
      const float cq = c[q0 + qq];
#pragma unroll
      for (int r = 0; r < R; ++r) out[r] = fmaf(v[r + qq], cq, out[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = v[kPulseR + r];
  }
}

// Stores outputs kk .. kk + R - 1 of a row of n_t samples (16-byte stores
// when kVec and the block is whole).
template <bool kVec, int R = kPulseR>
__device__ __forceinline__ void fir_store(float* row, int kk, int n_t, const float out[R]) {
  if (kVec && kk + R <= n_t) {
#pragma unroll
    for (int r = 0; r < R; r += 4)
      *reinterpret_cast<float4*>(row + kk + r) = make_float4(out[r], out[r + 1], out[r + 2], out[r + 3]);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (kk + r < n_t) row[kk + r] = out[r];
  }
}

}  // namespace usrt
