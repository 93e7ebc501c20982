// Internal interface of the neural-operator surrogate (fno_gemm.hip, fno.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qla {
namespace fno {

// BF16 as raw 16-bit patterns: round to nearest even from FP32.
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(h) << 16);
}

// C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n] (+ C if beta) (+ bias[m]) (+ res[b][m][n]);
// if act, GELU of the stored value is also written (BF16) at act with C's strides;
// atomic: atomicAdd alpha * product into an FP32 C (no bias, res, beta or act).
// Operands are BF16 bit patterns; element (b, m, k) of A is A[b*sAb + m*sAm + k*sAk].
// The K range is split over ksplit blocks (only with atomic).
struct GemmDesc {
  const uint16_t* A = nullptr;
  long long sAb = 0, sAm = 0, sAk = 0;
  const uint16_t* B = nullptr;
  long long sBb = 0, sBk = 0, sBn = 0;
  void* C = nullptr;
  long long sCb = 0, sCm = 0, sCn = 0;
  int M = 0, N = 0, K = 0, batch = 1, ksplit = 1;
  float alpha = 1.0f;
  int beta = 0, atomic = 0, out_bf16 = 0;
  const float* bias = nullptr;
  const float* res = nullptr;
  long long sRb = 0, sRm = 0, sRn = 0;
  uint16_t* act = nullptr;
};

hipError_t launch_gemm(const GemmDesc& g, hipStream_t stream);

}  // namespace fno
}  // namespace qla
