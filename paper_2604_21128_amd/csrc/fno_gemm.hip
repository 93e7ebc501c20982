// Batched, strided BF16 GEMM on the gfx950 matrix cores (v_mfma_f32_32x32x16_bf16),
// FP32 accumulation, used for every contraction of the neural-operator surrogate:
// channel mixing (1x1 convolutions), the truncated Fourier transforms written as
// products with cosine/sine bases, and all of their backward products.
//
//   C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n]  (+ C)  (+ bias[m]) (+ R[b][m][n])
//
// Every operand is addressed through its own strides, so transposed operands are
// just swapped strides. A block computes a 64x64 tile of C with 4 waves (2x2 of
// 32x32), stepping K by 32 through LDS tiles stored k-contiguous for both operands
// (one 16-byte LDS read per MFMA operand). Global loads take a vector path when the
// operand is contiguous along k or along its free index, else a scalar path; all
// accesses are bounds-checked and out-of-range elements are zero.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fno_internal.h"

namespace qla {
namespace fno {

namespace {

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

// Loads the kBM x kBK tile of a "row" operand (A: rows m; B seen as rows n) into
// lds[r][k] (k contiguous). Element (r, k) of the operand is at p[r * sr + k * sk].
__device__ __forceinline__ void load_tile(uint16_t (*lds)[kBK + kPad], const uint16_t* p,
                                          long long sr, long long sk, int r0, int rmax,
                                          int k0, int kmax) {
  const int t = threadIdx.x;
  if (sk == 1) {
    // 64 rows x 4 groups of 8 consecutive k
    const int r = t >> 2, kg = (t & 3) * 8;
    const int gr = r0 + r, gk = k0 + kg;
    uint16_t v[8];
    if (gr < rmax && gk + 8 <= kmax && (((reinterpret_cast<uintptr_t>(p + gr * sr + gk)) & 15) == 0)) {
      const uint4 w = *reinterpret_cast<const uint4*>(p + gr * sr + gk);
      __builtin_memcpy(v, &w, 16);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        v[i] = (gr < rmax && gk + i < kmax) ? p[gr * sr + gk + i] : uint16_t(0);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) lds[r][kg + i] = v[i];
  } else if (sr == 1) {
    // 32 k x 8 groups of 8 consecutive rows
    const int k = t >> 3, rg = (t & 7) * 8;
    const int gk = k0 + k, gr = r0 + rg;
    uint16_t v[8];
    if (gk < kmax && gr + 8 <= rmax && (((reinterpret_cast<uintptr_t>(p + gk * sk + gr)) & 15) == 0)) {
      const uint4 w = *reinterpret_cast<const uint4*>(p + gk * sk + gr);
      __builtin_memcpy(v, &w, 16);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        v[i] = (gk < kmax && gr + i < rmax) ? p[gk * sk + gr + i] : uint16_t(0);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) lds[rg + i][k] = v[i];
  } else {
    for (int e = t; e < kBM * kBK; e += 256) {
      const int r = e / kBK, k = e % kBK;
      const int gr = r0 + r, gk = k0 + k;
      lds[r][k] = (gr < rmax && gk < kmax) ? p[gr * sr + gk * sk] : uint16_t(0);
    }
  }
}

__global__ __launch_bounds__(256) void gemm_kernel(GemmDesc g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kBK + kPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kBK + kPad];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN;
  const int z = blockIdx.z;
  const int b = z / g.ksplit, split = z % g.ksplit;
  const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + kBK - 1) / kBK * kBK;
  const int kb = split * kchunk, ke = min(g.K, kb + kchunk);
  const uint16_t* A = g.A + b * g.sAb;
  const uint16_t* B = g.B + b * g.sBb;
  f32x16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += kBK) {
    load_tile(As, A, g.sAm, g.sAk, m0, g.M, k0, ke);
    load_tile(Bs, B, g.sBn, g.sBk, n0, g.N, k0, ke);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      const bf16x8 a =
          *reinterpret_cast<const bf16x8*>(&As[wm * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
      const bf16x8 bb =
          *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: accumulator 4i + j holds row 8i + 4(lane/32) + j, column lane % 32
  const int n = n0 + wn * 32 + (lane & 31);
  if (n >= g.N) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + wm * 32 + 8 * i + 4 * (lane >> 5) + j;
      if (m >= g.M) continue;
      float v = g.alpha * acc[4 * i + j];
      const long long co = b * g.sCb + m * g.sCm + n * g.sCn;
      if (g.atomic) {
        atomicAdd(static_cast<float*>(g.C) + co, v);
        continue;
      }
      if (g.bias) v += g.bias[m];
      if (g.res) v += g.res[b * g.sRb + m * g.sRm + n * g.sRn];
      if (g.out_bf16) {
        uint16_t* c = static_cast<uint16_t*>(g.C) + co;
        if (g.beta) v += bf16_to_f32(*c);
        *c = f32_to_bf16(v);
      } else {
        float* c = static_cast<float*>(g.C) + co;
        if (g.beta) v += *c;
        *c = v;
      }
      if (g.act) g.act[b * g.sCb + m * g.sCm + n * g.sCn] = f32_to_bf16(gelu(v));
    }
  }
}

}  // namespace

hipError_t launch_gemm(const GemmDesc& g, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0 || g.ksplit <= 0) return hipSuccess;
  // M tiles along x (no practical limit), N tiles and batch x split along y and z
  const long long ny = (g.N + kBN - 1) / kBN, nz = static_cast<long long>(g.batch) * g.ksplit;
  if (ny > 65535 || nz > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((g.M + kBM - 1) / kBM, static_cast<unsigned>(ny), static_cast<unsigned>(nz));
  hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, stream, g);
  return hipGetLastError();
}

}  // namespace fno
}  // namespace qla
