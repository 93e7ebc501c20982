// Internal interface of the neural-operator surrogate (fno_gemm.hip, fno.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qla {
namespace fno {

// BF16 as raw 16-bit patterns: round to nearest even from FP32. On the device the gfx950
// conversion instruction (v_cvt_pk_bf16_f32, two values per instruction) does it; on the
// host the same rounding is written out (finite values give the same bits).
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
#else
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
#endif
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(h) << 16);
}

// GELU(x) = x Phi(x) = (x / 2)(1 + erf(x / sqrt 2)) and GELU'(x) = Phi(x) + x phi(x), with
// erf from Abramowitz & Stegun, Handbook of Mathematical Functions, formula 7.1.26
// (|error| <= 1.5e-7, far below the BF16 rounding around them):
//   1 - erf(z) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-z^2), t = 1 / (1 + p z), z >= 0,
// odd in z. With z = |x| / sqrt 2 the same exp(-z^2) = exp(-x^2 / 2) gives the normal
// density phi(x) = exp(-x^2 / 2) / sqrt(2 pi), so the derivative costs one exponential (the
// hardware exp2) and one reciprocal. 1 - erf(|z|) is formed directly, so neither tail
// loses its relative accuracy to cancellation.
struct ErfTail {
  float c;  // 1 - erf(|x| / sqrt 2)
  float e;  // exp(-x^2 / 2)
};
__device__ __forceinline__ ErfTail erf_tail(float x) {
  const float z = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, z, 1.0f));
  float poly = 1.061405429f;
  poly = fmaf(poly, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  const float e = __builtin_amdgcn_exp2f(-z * z * 1.4426950408889634f);
  return {poly * t * e, e};
}
// x Phi(x) = max(x, 0) - |x| c / 2 for either sign (no select): for x >= 0 the same fused
// multiply-add as x - x c / 2, for x < 0 the one rounding of x c / 2.
__device__ __forceinline__ float gelu_as(float x) {
  const float c = erf_tail(x).c;
  return fmaf(-0.5f * fabsf(x), c, fmaxf(x, 0.0f));
}
__device__ __forceinline__ float gelu_prime_as(float x) {
  const ErfTail r = erf_tail(x);
  const float cdf = x >= 0.0f ? fmaf(-0.5f, r.c, 1.0f) : 0.5f * r.c;  // Phi(x)
  return fmaf(x * 0.39894228040143268f, r.e, cdf);
}

// C[b][m][n] = alpha * (sum_k A[b][m][k] B[b][k][n] + seg2) (+ bias[m]) (+ res[b][m][n])
//              (+ C if beta), then times GELU'(gz[b][m][n]) if gz;
// stored at C (BF16 or FP32) if C is set; if act, GELU of the value is also stored
// (BF16) at act with C's strides.
// seg2 (K2 > 0): a second contraction whose operands depend on the row and column of
// n = y * row + x in an H x row grid: sum_j A2[b][m][y][j] B2[j][x]. Needs
// row % 64 == 0 and ksplit == 1.
// atomic: atomicAdd alpha * product into an FP32 C (no bias, res, beta, gz or act).
// rowsum: also atomically add each row sum of A over k into rowsum[m] (blocks of
// the first column tile only; used for bias gradients).
// Operands are BF16 bit patterns; element (b, m, k) of A is A[b*sAb + m*sAm + k*sAk].
// The K range of the first contraction is split over ksplit blocks (only with atomic).
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
  const uint16_t* gz = nullptr;
  float* rowsum = nullptr;
  const uint16_t* A2 = nullptr;
  long long sA2b = 0, sA2m = 0, sA2y = 0, sA2k = 0;
  const uint16_t* B2 = nullptr;
  long long sB2k = 0, sB2x = 0;
  int K2 = 0, row = 0;
  int vec = 0;  // set by launch_gemm: 16-byte row stores in the epilogue
};

hipError_t launch_gemm(const GemmDesc& g, hipStream_t stream);

}  // namespace fno
}  // namespace qla
