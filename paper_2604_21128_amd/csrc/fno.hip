// Neural-operator surrogate of the QLA run: a Fourier neural operator (lift, L
// Fourier layers, two-layer projection) in BF16 storage with FP32 accumulation,
// trained and run entirely with this library's kernels (C ABI: qla_fno_* in qla.h).
//
// A Fourier layer maps v (C channels on an H x W periodic grid) to
//   act( IDFT[ R . DFT(v) ] + W v + b ),   act = GELU except after the last layer,
// where DFT keeps the modes ky in [0, m) U [H - m, H), kx in [0, m) of the 2D real
// transform and R mixes channels per mode with complex C x C weights. The truncated
// transforms are products with cosine/sine bases, done as BF16 GEMMs on the matrix
// cores (fno_gemm.hip):
//   x:   Z[(b,c,y)][2kx+p]   = sum_x v[(b,c,y)][x] Fx[x][2kx+p]       (p = re, im)
//   y:   T[(b,c)][2kyi+p][kx] = A1 . Zre + A2 . Zim                    (complex e^{-i..})
//   mix: S[(b,o)] = sum_c R[kyi][kx][c][o] T[(b,c)]                     (complex)
//   y^-1: U[(b,o)][y][2kx+p] = IY_p . S
//   x^-1: out[(b,o,y)][x]    = sum U Ix,  with weights 1 (kx = 0), 2 (kx > 0) and 1/(HW)
// which is the real inverse transform of the retained half spectrum. The backward pass
// uses the transposed products; gradients of the mode mixing and the pointwise parts
// are accumulated in FP32, and Adam updates FP32 master weights whose BF16 copies feed
// the GEMMs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fno_internal.h"
#include "qla.h"
#include "qla_ctx.h"

using qla::DeviceGuard;
using qla::fail;
using qla::hip_fail;
using qla::fno::bf16_to_f32;
using qla::fno::f32_to_bf16;
using qla::fno::GemmDesc;

namespace {

constexpr int kBlock = 256;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

using qla::fno::gelu_as;
using qla::fno::gelu_prime_as;

unsigned grid_for(size_t n) {
  const size_t b = (n + kBlock - 1) / kBlock;
  return static_cast<unsigned>(b < 16384 ? (b ? b : 1) : 16384);
}

__global__ void cast_kernel(const float* __restrict__ s, uint16_t* __restrict__ d, size_t n) {
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock)
    d[i] = f32_to_bf16(s[i]);
}

// Lift, v[b][c][p] = BF16(bp[c] + sum_i Wp[c][i] in[b][i][p]): with few input
// channels the product is a pure stream (read Cin, write C BF16 values per pixel), so
// it runs on the vector units: each thread takes 8 consecutive pixels, reads its
// inputs with 16-byte loads and writes each output channel's 8 values with one
// 16-byte store (a wavefront covers 1 KB of one channel's row per store).
// Weights are the BF16 copies the GEMM path uses. Shapes: Cin <= 8, C <= 256.
constexpr int kLiftMaxIn = 8, kLiftMaxC = 256;

__global__ __launch_bounds__(256) void lift_kernel(const uint16_t* __restrict__ in,
                                                   const uint16_t* __restrict__ w16,
                                                   const float* __restrict__ bias, int Cin,
                                                   int C, long long P, int B,
                                                   uint16_t* __restrict__ out) {
  __shared__ float sw[kLiftMaxC][kLiftMaxIn];
  __shared__ float sb[kLiftMaxC];
  for (int i = threadIdx.x; i < C * kLiftMaxIn; i += 256) {
    const int c = i / kLiftMaxIn, k = i % kLiftMaxIn;
    sw[c][k] = k < Cin ? bf16_to_f32(w16[c * Cin + k]) : 0.f;
  }
  for (int c = threadIdx.x; c < C; c += 256) sb[c] = bias[c];
  __syncthreads();
  const long long groups = (P + 7) / 8;  // 8-pixel groups per sample
  for (long long gi = blockIdx.x * 256LL + threadIdx.x; gi < groups * B;
       gi += static_cast<long long>(gridDim.x) * 256) {
    const int b = static_cast<int>(gi / groups);
    const long long p = (gi % groups) * 8;
    const bool full = p + 8 <= P;
    float x[kLiftMaxIn][8];
#pragma unroll
    for (int i = 0; i < kLiftMaxIn; ++i) {
      uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (i < Cin) {
        const uint16_t* src = in + (static_cast<long long>(b) * Cin + i) * P + p;
        if (full && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
          const uint4 q = *reinterpret_cast<const uint4*>(src);
          __builtin_memcpy(e, &q, 16);
        } else {
          for (int k = 0; k < 8; ++k) e[k] = p + k < P ? src[k] : uint16_t(0);
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) x[i][k] = bf16_to_f32(e[k]);
    }
    for (int c = 0; c < C; ++c) {
      uint16_t o[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        float a = sb[c];
#pragma unroll
        for (int i = 0; i < kLiftMaxIn; ++i) a = fmaf(sw[c][i], x[i][k], a);
        o[k] = f32_to_bf16(a);
      }
      uint16_t* dst = out + (static_cast<long long>(b) * C + c) * P + p;
      if (full && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        // non-temporal: the first layer reads it in a later launch
        __builtin_nontemporal_store(__builtin_bit_cast(u32x4_t, o), reinterpret_cast<u32x4_t*>(dst));
      } else {
        for (int k = 0; k < 8; ++k)
          if (p + k < P) dst[k] = o[k];
      }
    }
  }
}

// The second projection layer and its input gradient in training, where the product is
// narrow (Cout <= 4 output channels, C2 hidden ones) and a GEMM pads Cout to its tile:
// both are streams on the vector units, 8 consecutive pixels per thread (16-byte loads and
// stores), the weights (BF16 copies, as the GEMM path uses) and bias in LDS.
//   forward:  out[b][o][p] = bq2[o] + sum_h Q2[o][h] h[b][h][p]                 (FP32)
//   backward: dzq[b][h][p] = (sum_o Q2[o][h] dout[b][o][p]) GELU'(zq[b][h][p])  (BF16)
// Shapes: Cout <= kNarrowOut, C2 <= kNarrowC2, P a multiple of 8 (else the GEMM path).
constexpr int kNarrowOut = 4, kNarrowC2 = 256;

__device__ __forceinline__ void load8_bf16(const uint16_t* src, float* x) {
  const uint4 q = *reinterpret_cast<const uint4*>(src);
  uint16_t e[8];
  __builtin_memcpy(e, &q, 16);
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = bf16_to_f32(e[k]);
}

__global__ __launch_bounds__(256) void narrow_projection_kernel(
    const uint16_t* __restrict__ h, const uint16_t* __restrict__ q2,
    const float* __restrict__ bias, int C2, int Cout, long long P, int B,
    float* __restrict__ out) {
  __shared__ float sw[kNarrowOut][kNarrowC2];
  for (int i = threadIdx.x; i < kNarrowOut * kNarrowC2; i += 256) {
    const int o = i / kNarrowC2, c = i % kNarrowC2;
    sw[o][c] = (o < Cout && c < C2) ? bf16_to_f32(q2[o * C2 + c]) : 0.f;
  }
  __syncthreads();
  const long long groups = P / 8;
  for (long long gi = blockIdx.x * 256LL + threadIdx.x; gi < groups * B;
       gi += static_cast<long long>(gridDim.x) * 256) {
    const int b = static_cast<int>(gi / groups);
    const long long p = (gi % groups) * 8;
    float acc[kNarrowOut][8];
#pragma unroll
    for (int o = 0; o < kNarrowOut; ++o)
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[o][k] = o < Cout ? bias[o] : 0.f;
    const uint16_t* src = h + static_cast<long long>(b) * C2 * P + p;
    for (int c = 0; c < C2; ++c) {
      float x[8];
      load8_bf16(src + static_cast<long long>(c) * P, x);
#pragma unroll
      for (int o = 0; o < kNarrowOut; ++o)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[o][k] = fmaf(sw[o][c], x[k], acc[o][k]);
    }
    for (int o = 0; o < Cout; ++o) {
      float* dst = out + (static_cast<long long>(b) * Cout + o) * P + p;
      *reinterpret_cast<float4*>(dst) = make_float4(acc[o][0], acc[o][1], acc[o][2], acc[o][3]);
      *reinterpret_cast<float4*>(dst + 4) =
          make_float4(acc[o][4], acc[o][5], acc[o][6], acc[o][7]);
    }
  }
}

__global__ __launch_bounds__(256) void narrow_projection_grad_kernel(
    const uint16_t* __restrict__ dout, const uint16_t* __restrict__ q2,
    const uint16_t* __restrict__ zq, int C2, int Cout, long long P, int B,
    uint16_t* __restrict__ dzq) {
  __shared__ float sw[kNarrowC2][kNarrowOut];
  for (int i = threadIdx.x; i < kNarrowOut * kNarrowC2; i += 256) {
    const int c = i / kNarrowOut, o = i % kNarrowOut;
    sw[c][o] = (o < Cout && c < C2) ? bf16_to_f32(q2[o * C2 + c]) : 0.f;
  }
  __syncthreads();
  const long long groups = P / 8;
  for (long long gi = blockIdx.x * 256LL + threadIdx.x; gi < groups * B;
       gi += static_cast<long long>(gridDim.x) * 256) {
    const int b = static_cast<int>(gi / groups);
    const long long p = (gi % groups) * 8;
    float d[kNarrowOut][8];
#pragma unroll
    for (int o = 0; o < kNarrowOut; ++o) {
      if (o < Cout) {
        load8_bf16(dout + (static_cast<long long>(b) * Cout + o) * P + p, d[o]);
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) d[o][k] = 0.f;
      }
    }
    const long long base = static_cast<long long>(b) * C2 * P + p;
    for (int c = 0; c < C2; ++c) {
      float z[8];
      load8_bf16(zq + base + static_cast<long long>(c) * P, z);
      uint16_t e[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        float v = 0.f;
#pragma unroll
        for (int o = 0; o < kNarrowOut; ++o) v = fmaf(sw[c][o], d[o][k], v);
        e[k] = f32_to_bf16(v * gelu_prime_as(z[k]));
      }
      uint4 q;
      __builtin_memcpy(&q, e, 16);
      *reinterpret_cast<uint4*>(dzq + base + static_cast<long long>(c) * P) = q;
    }
  }
}

// Inference projection in one pass:
//   out[b][o][p] = bq2[o] + sum_h Q2[o][h] GELU(bq1[h] + sum_c Q1[h][c] v[b][c][p]).
// The C2-channel hidden layer never leaves the chip (the two-GEMM path writes it to
// HBM in BF16 and reads it back: 2 x 2 C2 bytes per pixel). Wave w owns hidden rows
// 32w .. 32w + 31 and keeps their Q1 fragments in registers; bq1 and Q2 sit in LDS.
// The block then strides over tiles of 64 pixels of one sample: the tile's channels
// go through LDS 32 at a time (each thread fetches 8 pixels of one channel, 16 bytes,
// and stores them pixel-major, 8-channel groups XORed with bits 3-4 of the pixel so
// the transposing stores spread over the banks), the waves multiply with the
// 32x32x16 BF16 matrix instruction (accumulator 4i + j = hidden row 8i + 4(lane/32)
// + j, pixel lane % 32), add the bias and apply GELU in FP32. The second projection runs
// on the matrix cores too, straight from those registers: accumulator registers 8m ..
// 8m + 7 of a lane hold hidden rows 16m + 4(lane/32) + {0..3, 8..11} of its pixel,
// exactly the 8 k slots a 32x32x16 B operand takes from that lane, so two products with
// Q2 fragments (rows: outputs, k slots in the same order of hidden rows) fold a wave's 32
// rows into the Cout output rows (GELU rounded to BF16 on the way, as the training path
// stores it); the waves' sums meet in LDS. Channels, rows and pixels beyond C, C2 and P
// are zero. Shapes: C <= 64, C2 <= 128, Cout <= 4 (else the two-GEMM path).
constexpr int kProjPix = 64, kProjK = 32, kProjMaxC = 64, kProjMaxC2 = 128, kProjMaxOut = 4;


// GELU in the fused kernels: the Abramowitz & Stegun form of fno_internal.h (with the
// library erff the GELUs were half of the projection kernel's time: every hidden value
// of every pixel).
__device__ __forceinline__ float gelu_f(float x) { return gelu_as(x); }

__device__ __forceinline__ int proj_col(int r, int k) {
  return ((((k >> 3) ^ (r >> 3)) & 3) << 3) | (k & 7);
}

__global__ __launch_bounds__(256) void projection_fused_kernel(
    const uint16_t* __restrict__ v, const uint16_t* __restrict__ q1,
    const float* __restrict__ bq1, const uint16_t* __restrict__ q2,
    const float* __restrict__ bq2, int C, int C2, int Cout, long long P, int B,
    float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t vs[kProjPix][kProjK + 8];
  __shared__ float red[4][kProjMaxOut][kProjPix];
  __shared__ float sb1[kProjMaxC2];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int hl = lane & 31, kh = 8 * (lane >> 5);
  for (int i = t; i < kProjMaxC2; i += 256) sb1[i] = i < C2 ? bq1[i] : 0.f;
  // Q2 fragments of this wave's hidden rows: output row hl, k slot e of product m is hidden
  // row 32 w + 8 (2 m + e / 4) + 4 (lane / 32) + e % 4 (the accumulator's row of register
  // 8 m + e)
  bf16x8_t q2f[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    uint16_t e8[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int h = 32 * w + 8 * (2 * m + e / 4) + 4 * (lane >> 5) + e % 4;
      e8[e] = (hl < Cout && h < C2) ? q2[hl * C2 + h] : uint16_t(0);
    }
    q2f[m] = __builtin_bit_cast(bf16x8_t, e8);
  }
  // this lane's A fragments: row 32w + hl of Q1, channels kc + kk + kh .. + 7
  const int hr = 32 * w + hl;
  bf16x8_t afr[kProjMaxC / 16];
#pragma unroll
  for (int f = 0; f < kProjMaxC / 16; ++f) {
    const int k = 16 * f + kh;
    uint16_t av[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      av[i] = (hr < C2 && k + i < C) ? q1[static_cast<long long>(hr) * C + k + i] : uint16_t(0);
    afr[f] = __builtin_bit_cast(bf16x8_t, av);
  }
  const int fk = t >> 3, fr = (t & 7) * 8;  // fetch: channel kc + fk, pixels fr .. fr + 7
  const long long tiles_per_sample = (P + kProjPix - 1) / kProjPix;
  const long long tiles = tiles_per_sample * B;
  for (long long tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int b = static_cast<int>(tile / tiles_per_sample);
    const long long p0 = (tile % tiles_per_sample) * kProjPix;
    const uint16_t* vb = v + static_cast<long long>(b) * C * P;
    f32x16_t acc0 = {}, acc1 = {};
#pragma unroll
    for (int kc = 0; kc < kProjMaxC; kc += kProjK) {
      if (kc >= C) break;
      uint16_t e[8];
      {
        const int c = kc + fk;
        const long long pp = p0 + fr;
        const uint16_t* src = vb + static_cast<long long>(c) * P + pp;
        if (c < C && pp + 8 <= P && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
          const uint4 q = *reinterpret_cast<const uint4*>(src);
          __builtin_memcpy(e, &q, 16);
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) e[i] = (c < C && pp + i < P) ? src[i] : uint16_t(0);
        }
      }
      __syncthreads();  // the previous tile has been read
#pragma unroll
      for (int i = 0; i < 8; ++i) vs[fr + i][proj_col(fr + i, fk)] = e[i];
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kProjK; kk += 16) {
        const int kg = kk + kh;
        const bf16x8_t b0 = *reinterpret_cast<const bf16x8_t*>(&vs[hl][proj_col(hl, kg)]);
        const bf16x8_t b1 =
            *reinterpret_cast<const bf16x8_t*>(&vs[32 + hl][proj_col(32 + hl, kg)]);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr[(kc + kk) / 16], b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr[(kc + kk) / 16], b1, acc1, 0, 0, 0);
      }
    }
    f32x16_t o0 = {}, o1 = {};
    if (32 * w < C2) {
      uint16_t g0[16], g1[16];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float bias = sb1[32 * w + 8 * i + 4 * (lane >> 5) + j];  // < kProjMaxC2
          g0[4 * i + j] = f32_to_bf16(gelu_f(acc0[4 * i + j] + bias));
          g1[4 * i + j] = f32_to_bf16(gelu_f(acc1[4 * i + j] + bias));
        }
      }
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        bf16x8_t b0, b1;
        __builtin_memcpy(&b0, g0 + 8 * m, 16);
        __builtin_memcpy(&b1, g1 + 8 * m, 16);
        o0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(q2f[m], b0, o0, 0, 0, 0);
        o1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(q2f[m], b1, o1, 0, 0, 0);
      }
    }
    // output row o of the products: register o of lanes 0 .. 31 (o < 4), pixel lane
    if (lane < 32) {
#pragma unroll
      for (int o = 0; o < kProjMaxOut; ++o) {
        red[w][o][lane] = o0[o];
        red[w][o][32 + lane] = o1[o];
      }
    }
    __syncthreads();
    for (int idx = t; idx < Cout * kProjPix; idx += 256) {
      const int o = idx / kProjPix, px = idx % kProjPix;
      const long long pp = p0 + px;
      if (pp >= P) continue;
      const float sum = bq2[o] + red[0][o][px] + red[1][o][px] + red[2][o][px] + red[3][o][px];
      out[(static_cast<long long>(b) * Cout + o) * P + pp] = sum;
    }
    // red and vs are rewritten only after the next tile's first barrier
  }
}

// Pointwise + spectral part of a Fourier layer for C = 64 channels on rows of a
// multiple of 256 pixels:
//   pre[b][o][p] = bias[o] + sum_c Wl[o][c] v[b][c][p] + sum_j U[b][o][y][j] IX[j][x]
// (p = y W + x; the second sum is the inverse x transform of the spectral branch),
// stored as BF16 pre-activation (zout, optional) and BF16 GELU(pre) (aout, optional).
// The generic GEMM does this with 64-pixel tiles, i.e. 128-byte runs per channel row;
// here a block strides over tiles of 256 pixels of one grid row (512-byte runs, 1 KB
// per wavefront load or store). The tile's 64 channels go to LDS pixel-major (8-channel
// groups XORed with bits 3-5 of the pixel), the 256 columns of IX likewise; the 4
// waves (2 x 2) each compute 32 output channels x 128 pixels with the 32x32x16 BF16
// matrix instruction, Wl fragments held in registers for the block's lifetime; the
// next tile's loads are issued before the current tile's products; outputs are staged
// in LDS and written row by row with 16-byte stores. v is read and the outputs written
// with the non-temporal policy (streamed once each; 331 -> 320 us per 512^2 layer of
// batch 16).
constexpr int kMixC = 64, kMixPix = 256, kMixMaxJ = 32;

__device__ __forceinline__ int mix_col64(int r, int k) {
  return ((((k >> 3) ^ (r >> 3)) & 7) << 3) | (k & 7);
}
__device__ __forceinline__ int mix_col32(int r, int k) {
  return ((((k >> 3) ^ (r >> 3)) & 3) << 3) | (k & 7);
}

// kBack = false: the forward layer above. kBack = true: its input-gradient product with
// the same tiling, roles and operands in the same places,
//   out[b][c][p] = (sum_o Wl[o][c] dz[b][o][p] + sum_j dZ[b][c][y][j] Fx[x][j]) GELU'(gz)
// (v = dz, U = dZ, the LDS basis slice Fx instead of IX, no bias; without gz the factor is
// 1), the sums staged in LDS in FP32 (32 rows at a time) so the factor multiplies the
// FP32 value, as the GEMM epilogue does.
template <bool kBack>
__global__ __launch_bounds__(256) void layer_mix_kernel(
    const uint16_t* __restrict__ v, const uint16_t* __restrict__ wl,
    const float* __restrict__ bias, const uint16_t* __restrict__ U,
    const uint16_t* __restrict__ IX, int m2, int H, int W, int B,
    uint16_t* __restrict__ zout, uint16_t* __restrict__ aout, const uint16_t* __restrict__ gz) {
  // v tile [pixel][channel]; after the products the same bytes stage the output rows
  __shared__ __attribute__((aligned(16))) uint16_t vs[kMixPix * (kMixC + 8)];
  __shared__ __attribute__((aligned(16))) uint16_t xs[kMixPix][kMixMaxJ + 8];
  __shared__ float sbias[kMixC];
  uint16_t(*ost)[kMixPix + 8] = reinterpret_cast<uint16_t(*)[kMixPix + 8]>(vs);
  float(*fst)[kMixPix + 4] = reinterpret_cast<float(*)[kMixPix + 4]>(vs);  // 32 rows, FP32
  static_assert(sizeof(float) * 32 * (kMixPix + 4) <= sizeof(uint16_t) * kMixPix * (kMixC + 8),
                "half the FP32 output rows fit where the tile was");
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
  const int hl = lane & 31, kh = 8 * (lane >> 5);
  const long long P = static_cast<long long>(H) * W;
  if (!kBack && t < kMixC) sbias[t] = bias[t];
  // weight fragments: row 32 wm + hl, k = 16 f + kh .. + 7 of Wl (forward: Wl[row][k]) or
  // of Wl^T (Wl[k][row])
  bf16x8_t afr[kMixC / 16];
#pragma unroll
  for (int f = 0; f < kMixC / 16; ++f) {
    if constexpr (kBack) {
      uint16_t e[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) e[i] = wl[(16 * f + kh + i) * kMixC + 32 * wm + hl];
      afr[f] = __builtin_bit_cast(bf16x8_t, e);
    } else {
      afr[f] = *reinterpret_cast<const bf16x8_t*>(wl + (32 * wm + hl) * kMixC + 16 * f + kh);
    }
  }
  const int per_row = W / kMixPix;
  const long long tiles = static_cast<long long>(B) * H * per_row;
  // The grid is a multiple of per_row (the launch makes it so), so all of this block's
  // tiles start at the same column x0: its 256 columns of the x basis (IX[j][x], or
  // Fx[x][j] backward) go into LDS once.
  {
    const int x0 = static_cast<int>(blockIdx.x % per_row) * kMixPix;
    if constexpr (kBack) {
      for (int idx = t; idx < kMixPix * kMixMaxJ; idx += 256) {
        const int r = idx / kMixMaxJ, j = idx % kMixMaxJ;
        xs[r][mix_col32(r, j)] = j < m2 ? IX[static_cast<long long>(x0 + r) * m2 + j] : uint16_t(0);
      }
    } else {
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int idx = it * 256 + t, j = idx >> 5, seg = idx & 31;
        const uint4 q = j < m2 ? *reinterpret_cast<const uint4*>(IX + static_cast<long long>(j) * W + x0 + seg * 8)
                               : uint4{0, 0, 0, 0};
        uint16_t e[8];
        __builtin_memcpy(e, &q, 16);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int r = seg * 8 + i;
          xs[r][mix_col32(r, j)] = e[i];
        }
      }
    }
  }
  // loads of one tile: 8 x 16 bytes of v per thread (channel idx >> 5, pixels
  // (idx & 31) * 8 ..)
  uint4 rv[8];
  auto load_tile = [&](long long tile) {
    const int b = static_cast<int>(tile / (static_cast<long long>(H) * per_row));
    const long long rem = tile % (static_cast<long long>(H) * per_row);
    const int y = static_cast<int>(rem / per_row), x0 = static_cast<int>(rem % per_row) * kMixPix;
    const uint16_t* vb = v + static_cast<long long>(b) * kMixC * P + static_cast<long long>(y) * W + x0;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = it * 256 + t, c = idx >> 5, seg = idx & 31;
      rv[it] = __builtin_bit_cast(
          uint4, __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(vb + c * P + seg * 8)));
    }
  };
  long long tile = blockIdx.x;
  if (tile < tiles) load_tile(tile);
  for (; tile < tiles; tile += gridDim.x) {
    const int b = static_cast<int>(tile / (static_cast<long long>(H) * per_row));
    const long long rem = tile % (static_cast<long long>(H) * per_row);
    const int y = static_cast<int>(rem / per_row), x0 = static_cast<int>(rem % per_row) * kMixPix;
    // U fragments of this tile's grid row: row 32 wm + hl, modes kh .. kh + 7 and 16 + kh ..
    // (16-byte loads when 2m is a multiple of 8: each group of 8 modes then lies wholly in or
    // out of the row, and rows start 16-byte aligned)
    bf16x8_t a2[2];
    const uint16_t* usrc = U + ((static_cast<long long>(b) * kMixC + 32 * wm + hl) * H + y) * m2;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const int j0 = 16 * f + kh;
      if (m2 % 8 == 0) {
        a2[f] = j0 < m2 ? *reinterpret_cast<const bf16x8_t*>(usrc + j0) : bf16x8_t{};
      } else {
        uint16_t e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = j0 + i < m2 ? usrc[j0 + i] : uint16_t(0);
        a2[f] = __builtin_bit_cast(bf16x8_t, e);
      }
    }
    __syncthreads();  // the previous tile's output staging has been read
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = it * 256 + t, c = idx >> 5, seg = idx & 31;
      uint16_t e[8];
      __builtin_memcpy(e, &rv[it], 16);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = seg * 8 + i;
        vs[r * (kMixC + 8) + mix_col64(r, c)] = e[i];
      }
    }
    __syncthreads();
    if (tile + gridDim.x < tiles) load_tile(tile + gridDim.x);  // in flight during the products
    // backward: GELU'(z) of the first 32 output rows, in flight during the products (the
    // second 32 rows' are loaded before their half of the epilogue)
    u32x4_t gq[4];
    const uint16_t* gb = nullptr;
    if constexpr (kBack) {
      if (gz) {
        gb = gz + static_cast<long long>(b) * kMixC * P + static_cast<long long>(y) * W + x0;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int idx = it * 256 + t, rr = idx >> 5, seg = idx & 31;
          gq[it] = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(gb + rr * P + seg * 8));
        }
      }
    }
    f32x16_t acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      acc[nt] = f32x16_t{};
      const int r = wn * 128 + nt * 32 + hl;
#pragma unroll
      for (int f = 0; f < kMixC / 16; ++f) {
        const bf16x8_t bb =
            *reinterpret_cast<const bf16x8_t*>(&vs[r * (kMixC + 8) + mix_col64(r, 16 * f + kh)]);
        acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr[f], bb, acc[nt], 0, 0, 0);
      }
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const bf16x8_t bb = *reinterpret_cast<const bf16x8_t*>(&xs[r][mix_col32(r, 16 * f + kh)]);
        acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[f], bb, acc[nt], 0, 0, 0);
      }
    }
    if constexpr (kBack) {
      // the FP32 sums, 32 rows at a time, times GELU'(gz), stored BF16
      uint16_t* db = zout + static_cast<long long>(b) * kMixC * P + static_cast<long long>(y) * W + x0;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        if (half == 1 && gb) {
#pragma unroll
          for (int it = 0; it < 4; ++it) {
            const int idx = it * 256 + t, rr = idx >> 5, seg = idx & 31;
            gq[it] = __builtin_nontemporal_load(
                reinterpret_cast<const u32x4_t*>(gb + (32 + rr) * P + seg * 8));
          }
        }
        __syncthreads();  // the tile (or the previous half) is no longer read
        if (wm == half) {
#pragma unroll
          for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                fst[8 * i + 4 * (lane >> 5) + j][wn * 128 + nt * 32 + hl] = acc[nt][4 * i + j];
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int idx = it * 256 + t, rr = idx >> 5, seg = idx & 31, row = 32 * half + rr;
          const f32x4_t lo = *reinterpret_cast<const f32x4_t*>(&fst[rr][seg * 8]);
          const f32x4_t hi = *reinterpret_cast<const f32x4_t*>(&fst[rr][seg * 8 + 4]);
          uint16_t gv[8];
          if (gb) __builtin_memcpy(gv, &gq[it], 16);
          uint16_t e[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            float val = i < 4 ? lo[i] : hi[i - 4];
            if (gb) val *= gelu_prime_as(bf16_to_f32(gv[i]));
            e[i] = f32_to_bf16(val);
          }
          __builtin_nontemporal_store(__builtin_bit_cast(u32x4_t, e),
                                      reinterpret_cast<u32x4_t*>(db + row * P + seg * 8));
        }
      }
      continue;
    }
    // outputs: pre-activation, then GELU, each staged in LDS and stored row by row
    uint16_t* outs[2] = {zout, aout};
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      uint16_t* dst = outs[pass];
      if (!dst) continue;
      __syncthreads();  // the tile (or the previous pass) is no longer read
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int row = 32 * wm + 8 * i + 4 * (lane >> 5) + j;
            const float val = acc[nt][4 * i + j] + sbias[row];
            ost[row][wn * 128 + nt * 32 + hl] = f32_to_bf16(pass ? gelu_f(val) : val);
          }
        }
      }
      __syncthreads();
      uint16_t* db = dst + static_cast<long long>(b) * kMixC * P + static_cast<long long>(y) * W + x0;
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int idx = it * 256 + t, row = idx >> 5, seg = idx & 31;
        __builtin_nontemporal_store(*reinterpret_cast<const u32x4_t*>(&ost[row][seg * 8]),
                                    reinterpret_cast<u32x4_t*>(db + row * P + seg * 8));
      }
    }
  }
}

// Training's first projection, zq = Q1 v + bq1 and h = GELU(zq), for 64 input and 64 G
// output channels (G = 1 or 2) on rows of a multiple of 256 cells: a block takes 256-pixel
// tiles of grid rows in turn, stages each tile once in LDS ([pixel][channel], the layer
// kernel's swizzle, the next tile in flight) and multiplies it by each 64-row group of Q1;
// a group's outputs go through a staging buffer of their own (the tile stays for the next
// group) and are stored row by row with 16-byte non-temporal stores. The GEMM it replaces
// read v once per 64 output channels through 64-pixel tiles. With out set (Cout <=
// kNarrowOut) the second projection, out = Q2 h + bq2, is formed from the staged BF16 h as
// narrow_projection_kernel forms it (bias first, then one FMA per hidden channel in order:
// the same bits), so h is not read back from memory; thread t takes pixel t of the tile.
constexpr int kProj1MaxGroups = 2;
__global__ __launch_bounds__(256, 2) void proj1_train_kernel(
    const uint16_t* __restrict__ v, const uint16_t* __restrict__ q1,
    const float* __restrict__ bias, int groups, int H, int W, int B, uint16_t* __restrict__ zq,
    uint16_t* __restrict__ hout, const uint16_t* __restrict__ q2,
    const float* __restrict__ bias2, int Cout, float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t vs[kMixPix * (kMixC + 8)];
  __shared__ __attribute__((aligned(16))) uint16_t ost[kMixC][kMixPix + 8];
  __shared__ float sbias[kProj1MaxGroups * kMixC];
  __shared__ float sw2[kNarrowOut][kProj1MaxGroups * kMixC];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
  const int hl = lane & 31, kh = 8 * (lane >> 5);
  const long long P = static_cast<long long>(H) * W;
  const int nout = groups * kMixC;
  if (t < nout) sbias[t] = bias[t];
  if (out) {
    for (int i = t; i < kNarrowOut * kProj1MaxGroups * kMixC; i += 256) {
      const int o = i / (kProj1MaxGroups * kMixC), c = i % (kProj1MaxGroups * kMixC);
      sw2[o][c] = (o < Cout && c < nout) ? bf16_to_f32(q2[o * nout + c]) : 0.f;
    }
  }
  // Q1 fragments of each group: row 64 g + 32 wm + hl, k = 16 f + kh .. + 7
  bf16x8_t afr[kProj1MaxGroups][kMixC / 16];
#pragma unroll
  for (int g = 0; g < kProj1MaxGroups; ++g)
#pragma unroll
    for (int f = 0; f < kMixC / 16; ++f)
      afr[g][f] = g < groups ? *reinterpret_cast<const bf16x8_t*>(
                                   q1 + (kMixC * g + 32 * wm + hl) * kMixC + 16 * f + kh)
                             : bf16x8_t{};
  const int per_row = W / kMixPix;
  const long long tiles = static_cast<long long>(B) * H * per_row;
  uint4 rv[8];
  auto load_tile = [&](long long tile) {
    const int b = static_cast<int>(tile / (static_cast<long long>(H) * per_row));
    const long long rem = tile % (static_cast<long long>(H) * per_row);
    const int y = static_cast<int>(rem / per_row), x0 = static_cast<int>(rem % per_row) * kMixPix;
    const uint16_t* vb = v + static_cast<long long>(b) * kMixC * P + static_cast<long long>(y) * W + x0;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = it * 256 + t, c = idx >> 5, seg = idx & 31;
      rv[it] = __builtin_bit_cast(
          uint4, __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(vb + c * P + seg * 8)));
    }
  };
  long long tile = blockIdx.x;
  if (tile < tiles) load_tile(tile);
  for (; tile < tiles; tile += gridDim.x) {
    const int b = static_cast<int>(tile / (static_cast<long long>(H) * per_row));
    const long long rem = tile % (static_cast<long long>(H) * per_row);
    const int y = static_cast<int>(rem / per_row), x0 = static_cast<int>(rem % per_row) * kMixPix;
    __syncthreads();  // the previous tile is no longer read
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = it * 256 + t, c = idx >> 5, seg = idx & 31;
      uint16_t e[8];
      __builtin_memcpy(e, &rv[it], 16);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = seg * 8 + i;
        vs[r * (kMixC + 8) + mix_col64(r, c)] = e[i];
      }
    }
    __syncthreads();
    if (tile + gridDim.x < tiles) load_tile(tile + gridDim.x);  // in flight during the products
    float oacc[kNarrowOut];
#pragma unroll
    for (int o = 0; o < kNarrowOut; ++o) oacc[o] = (out && o < Cout) ? bias2[o] : 0.f;
    for (int g = 0; g < groups; ++g) {
      f32x16_t acc[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        acc[nt] = f32x16_t{};
        const int r = wn * 128 + nt * 32 + hl;
#pragma unroll
        for (int f = 0; f < kMixC / 16; ++f) {
          const bf16x8_t bb =
              *reinterpret_cast<const bf16x8_t*>(&vs[r * (kMixC + 8) + mix_col64(r, 16 * f + kh)]);
          acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(g ? afr[1][f] : afr[0][f], bb,
                                                            acc[nt], 0, 0, 0);
        }
      }
      // pre-activation, then GELU, each staged in LDS and stored row by row
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        __syncthreads();  // the staging buffer is no longer read
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int row = 32 * wm + 8 * i + 4 * (lane >> 5) + j;
              const float val = acc[nt][4 * i + j] + sbias[kMixC * g + row];
              ost[row][wn * 128 + nt * 32 + hl] = f32_to_bf16(pass ? gelu_f(val) : val);
            }
        __syncthreads();
        uint16_t* db = (pass ? hout : zq) +
                       (static_cast<long long>(b) * nout + kMixC * g) * P +
                       static_cast<long long>(y) * W + x0;
#pragma unroll
        for (int it = 0; it < 8; ++it) {
          const int idx = it * 256 + t, row = idx >> 5, seg = idx & 31;
          __builtin_nontemporal_store(*reinterpret_cast<const u32x4_t*>(&ost[row][seg * 8]),
                                      reinterpret_cast<u32x4_t*>(db + row * P + seg * 8));
        }
        // the second projection's share of this group's channels, while the stores drain
        if (pass == 1 && out) {
          for (int r = 0; r < kMixC; ++r) {
            const float x = bf16_to_f32(ost[r][t]);
#pragma unroll
            for (int o = 0; o < kNarrowOut; ++o) oacc[o] = fmaf(sw2[o][kMixC * g + r], x, oacc[o]);
          }
        }
      }
    }
    if (out) {
#pragma unroll
      for (int o = 0; o < kNarrowOut; ++o)
        if (o < Cout)
          out[(static_cast<long long>(b) * Cout + o) * P + static_cast<long long>(y) * W + x0 +
              t] = oacc[o];
    }
  }
}

// Backward through training's two projections in one pass over zq (64 input channels, 64 G
// hidden channels with G = 1 or 2, Cout <= kNarrowOut outputs, rows of a multiple of 256
// cells):
//   dzq[b][h][p] = GELU'(zq[b][h][p]) sum_o Q2[o][h] dout[b][o][p]  (stored: the first
//                  projection's weight gradient reads it),
//   dz[b][c][p]  = sum_h Q1[h][c] dzq[b][h][p].
// dzq is formed as narrow_projection_grad_kernel forms it (the same bits) and goes
// straight into the product's LDS tile ([pixel][channel], the layer kernel's swizzle), 64
// hidden channels at a time, the next group's zq in flight during the products; the GEMM
// this replaces read dzq back from memory. dz is staged in the same LDS and stored row by
// row with 16-byte non-temporal stores.
__global__ __launch_bounds__(256, 2) void proj_grad_kernel(
    const uint16_t* __restrict__ dout, const uint16_t* __restrict__ q2,
    const uint16_t* __restrict__ zq, const uint16_t* __restrict__ q1, int groups, int Cout,
    int H, int W, int B, uint16_t* __restrict__ dzq, uint16_t* __restrict__ dz) {
  __shared__ __attribute__((aligned(16))) uint16_t vs[kMixPix * (kMixC + 8)];
  __shared__ float sw[kProj1MaxGroups * kMixC][kNarrowOut];
  uint16_t(*ost)[kMixPix + 8] = reinterpret_cast<uint16_t(*)[kMixPix + 8]>(vs);
  static_assert(kMixC * (kMixPix + 8) <= kMixPix * (kMixC + 8), "dz staging fits the tile");
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
  const int hl = lane & 31, kh = 8 * (lane >> 5), seg = t & 31;
  const long long P = static_cast<long long>(H) * W;
  const int C2 = groups * kMixC;
  for (int i = t; i < kProj1MaxGroups * kMixC * kNarrowOut; i += 256) {
    const int c = i / kNarrowOut, o = i % kNarrowOut;
    sw[c][o] = (o < Cout && c < C2) ? bf16_to_f32(q2[o * C2 + c]) : 0.f;
  }
  // Q1^T fragments of each group: row c = 32 wm + hl, k = h = 64 g + 16 f + kh .. + 7
  bf16x8_t afr[kProj1MaxGroups][kMixC / 16];
#pragma unroll
  for (int g = 0; g < kProj1MaxGroups; ++g)
#pragma unroll
    for (int f = 0; f < kMixC / 16; ++f) {
      uint16_t e[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        e[i] = g < groups ? q1[(kMixC * g + 16 * f + kh + i) * kMixC + 32 * wm + hl] : uint16_t(0);
      afr[g][f] = __builtin_bit_cast(bf16x8_t, e);
    }
  const int per_row = W / kMixPix;
  const long long tiles = static_cast<long long>(B) * H * per_row;
  auto tile_at = [&](long long tile, int* b, int* y, int* x0) {
    *b = static_cast<int>(tile / (static_cast<long long>(H) * per_row));
    const long long rem = tile % (static_cast<long long>(H) * per_row);
    *y = static_cast<int>(rem / per_row);
    *x0 = static_cast<int>(rem % per_row) * kMixPix;
  };
  // zq of one group of one tile: 8 x 16 bytes per thread (channel 64 g + (idx >> 5), the
  // thread's 8 pixels seg * 8 ..)
  uint4 rz[8];
  auto load_z = [&](long long tile, int g) {
    int b, y, x0;
    tile_at(tile, &b, &y, &x0);
    const uint16_t* zb = zq + (static_cast<long long>(b) * C2 + kMixC * g) * P +
                         static_cast<long long>(y) * W + x0 + seg * 8;
#pragma unroll
    for (int it = 0; it < 8; ++it)
      rz[it] = __builtin_bit_cast(uint4, __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(
                                             zb + ((it * 256 + t) >> 5) * P)));
  };
  long long tile = blockIdx.x;
  if (tile < tiles) load_z(tile, 0);
  for (; tile < tiles; tile += gridDim.x) {
    int b, y, x0;
    tile_at(tile, &b, &y, &x0);
    const long long pix = static_cast<long long>(y) * W + x0 + seg * 8;
    float d[kNarrowOut][8];
#pragma unroll
    for (int o = 0; o < kNarrowOut; ++o) {
      if (o < Cout) {
        load8_bf16(dout + (static_cast<long long>(b) * Cout + o) * P + pix, d[o]);
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) d[o][k] = 0.f;
      }
    }
    f32x16_t acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x16_t{};
    for (int g = 0; g < groups; ++g) {
      __syncthreads();  // the tile (previous group's, or previous tile's dz staging) is free
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int c = (it * 256 + t) >> 5, h = kMixC * g + c;
        uint16_t zv[8], e[8];
        __builtin_memcpy(zv, &rz[it], 16);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          float v = 0.f;
#pragma unroll
          for (int o = 0; o < kNarrowOut; ++o) v = fmaf(sw[h][o], d[o][k], v);
          e[k] = f32_to_bf16(v * gelu_prime_as(bf16_to_f32(zv[k])));
        }
        __builtin_nontemporal_store(__builtin_bit_cast(u32x4_t, e),
                                    reinterpret_cast<u32x4_t*>(
                                        dzq + (static_cast<long long>(b) * C2 + h) * P + pix));
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int r = seg * 8 + i;
          vs[r * (kMixC + 8) + mix_col64(r, c)] = e[i];
        }
      }
      __syncthreads();
      // the next group's (or the next tile's first group's) zq, in flight during the products
      if (g + 1 < groups) {
        load_z(tile, g + 1);
      } else if (tile + gridDim.x < tiles) {
        load_z(tile + gridDim.x, 0);
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int r = wn * 128 + nt * 32 + hl;
#pragma unroll
        for (int f = 0; f < kMixC / 16; ++f) {
          const bf16x8_t bb =
              *reinterpret_cast<const bf16x8_t*>(&vs[r * (kMixC + 8) + mix_col64(r, 16 * f + kh)]);
          acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(g ? afr[1][f] : afr[0][f], bb,
                                                            acc[nt], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // the last group's tile is no longer read
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = 32 * wm + 8 * i + 4 * (lane >> 5) + j;
          ost[row][wn * 128 + nt * 32 + hl] = f32_to_bf16(acc[nt][4 * i + j]);
        }
    __syncthreads();
    uint16_t* db = dz + static_cast<long long>(b) * kMixC * P + static_cast<long long>(y) * W + x0;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = it * 256 + t, row = idx >> 5, sg = idx & 31;
      __builtin_nontemporal_store(*reinterpret_cast<const u32x4_t*>(&ost[row][sg * 8]),
                                  reinterpret_cast<u32x4_t*>(db + row * P + sg * 8));
    }
  }
}

// The x and y transforms of a Fourier layer in one pass over v (grids of rows a multiple
// of 32 cells, widths a multiple of 128 up to 512 cells, m <= 16 modes):
//   T[(b,c)][r][kx] = sum_y A1[r][y] Z[y][2kx] + A2[r][y] Z[y][2kx+1],
//   Z[y][j]         = sum_x v[(b,c)][y][x] Fx[x][j],
// with Z rounded to BF16 as the separate transforms store it, but never written to
// memory. One block of 8 waves per plane (b, c) walks the plane in tiles of 32 whole
// rows, a contiguous 32 W x 2 bytes of memory read 1 KB per wave load instruction, with
// the non-temporal policy (v is read once; measured 135 -> 107 us per 512^2 layer of
// batch 16 against default loads); the next tile is in flight while one is worked on. A tile goes through LDS; wave w
// multiplies its 64-column slices (w, w + 8, ...) with the matching slices of the
// transposed basis FxT (2m rows, held in LDS for the block) on the matrix cores (32 x 32 x 16 BF16 products, FP32 accumulation), so each
// wave holds part of the tile's 32 x 2m product Z. The 8 parts meet in LDS (FP32, summed
// in wave order, then rounded to BF16), and each wave takes one 32 x 32 x 16 product of
// the y transform: rows 32 (w % 2) .. of T, tile rows 16 ((w / 2) % 2) .., and the real
// (w < 4: A1 with Z's columns 2kx) or imaginary part (A2 with columns 2kx + 1), with the
// tile's 32 columns of A1 and A2 staged in LDS beside it. At the end the 8 waves' parts of
// T are summed in a fixed order.
constexpr int kSpecCols = 32;   // Z columns: 2m <= 32
constexpr int kSpecRows = 64;   // T rows: 4m <= 64
constexpr int kSpecMaxW = 512;
constexpr int kSpecWaves = 8;
constexpr int kSpecZp = 36;     // column pitch (floats) of the FP32 parts of Z in LDS

struct SpecLds {
  int basis, tile, zred, aslc, total;  // byte offsets and size
};

__host__ __device__ inline SpecLds spec_lds_layout(int W, int m) {
  SpecLds L;
  const int ld = W + 8;
  L.basis = 0;
  L.tile = (2 * m * ld * 2 + 15) / 16 * 16;
  const int tile_bytes = 32 * ld * 2;
  const int zred_bytes = kSpecWaves * 2 * m * kSpecZp * 4;
  L.zred = L.tile;  // the FP32 parts of Z reuse the tile once it has been multiplied
  L.aslc = L.tile + (tile_bytes > zred_bytes ? tile_bytes : zred_bytes);
  L.total = L.aslc + 2 * 4 * m * 40 * 2;
  const int red = kSpecWaves * 32 * 16 * 4;  // the waves' parts of T, at the end
  if (L.total < red) L.total = red;
  return L;
}

size_t spectral_in_lds(int W, int m) { return static_cast<size_t>(spec_lds_layout(W, m).total); }

bool spectral_in_fits(int H, int W, int m) {
  return H % 32 == 0 && W % 128 == 0 && W <= kSpecMaxW && m >= 1 && 2 * m <= kSpecCols &&
         4 * m <= kSpecRows;
}

template <int NU, bool kModeMajor>
__global__ __launch_bounds__(64 * kSpecWaves, 4) void spectral_in_kernel(
    const uint16_t* __restrict__ v, long long sample_stride, long long plane_stride,
    int planes_per_sample, const uint16_t* __restrict__ fxt, const uint16_t* __restrict__ a1,
    const uint16_t* __restrict__ a2, int H, int W, int m, float* __restrict__ T) {
  extern __shared__ __attribute__((aligned(16))) char spec_smem[];
  constexpr int kThreads = 64 * kSpecWaves;
  const SpecLds L = spec_lds_layout(W, m);
  uint16_t* basis = reinterpret_cast<uint16_t*>(spec_smem + L.basis);  // [2m][W + 8]
  uint16_t* tile = reinterpret_cast<uint16_t*>(spec_smem + L.tile);    // [32][W + 8]
  float* zred = reinterpret_cast<float*>(spec_smem + L.zred);          // [wave][2m][36]
  uint16_t* aslc = reinterpret_cast<uint16_t*>(spec_smem + L.aslc);    // [part][4m][40]
  const int ld = W + 8;
  const int t = threadIdx.x, lane = t & 63, l32 = lane & 31, h = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  const int m2 = 2 * m, r4 = 4 * m, segs = W / 8;
  // the basis: at most 2m W / 8 / 512 <= 4 pieces of 16 bytes per thread (loads issued
  // for all four, past the end a spare copy of the last, so their count is fixed)
  constexpr int kBasisPieces = 4;
  const int nbp = m2 * segs;
  u32x4_t bv[kBasisPieces];
#pragma unroll
  for (int i = 0; i < kBasisPieces; ++i) {
    const int idx = min(t + i * kThreads, nbp - 1);
    bv[i] = *reinterpret_cast<const u32x4_t*>(fxt + static_cast<long long>(idx / segs) * W +
                                              (idx % segs) * 8);
  }
  const int b = blockIdx.x / planes_per_sample, c = blockIdx.x % planes_per_sample;
  const uint16_t* plane = v + b * sample_stride + c * plane_stride;
  const int tiles = H / 32;
  // this thread's share of loading a tile: the 16-byte pieces u 512 + t (u < W / 128) of
  // the tile's 32 W / 8 (a wave's load instruction reads 1 KB of consecutive rows), and,
  // for t < 2 * 4m * 4, the 16-byte piece of A1 or A2 at part t / 16m, row (t / 4) % 4m,
  // columns 8 (t % 4) .. of the tile's 32
  constexpr int nu = NU;  // W / 128
  int prow[NU], pcol[NU];
#pragma unroll
  for (int u = 0; u < nu; ++u) {
    prow[u] = (u * kThreads + t) / segs;
    pcol[u] = (u * kThreads + t) % segs * 8;
  }
  const bool has_a = t < 2 * r4 * 4;
  const int a_part = t / (4 * r4), a_row = (t / 4) % r4, a_col = 8 * (t % 4);
  const uint16_t* a_src = (a_part ? a2 : a1) + static_cast<long long>(has_a ? a_row : 0) * H + a_col;
  auto load = [&](u32x4_t(&rv)[NU], u32x4_t& av, int tl) {
    const uint16_t* p = plane + static_cast<long long>(tl) * 32 * W;
#pragma unroll
    for (int u = 0; u < nu; ++u)
      rv[u] = __builtin_nontemporal_load(
          reinterpret_cast<const u32x4_t*>(p + static_cast<long long>(prow[u]) * W + pcol[u]));
    av = *reinterpret_cast<const u32x4_t*>(a_src + tl * 32);  // (a spare copy if !has_a)
  };
  // wave w's share of the y transform: T rows 32 rt .., tile rows 16q .. (k slot 8h + i
  // is tile row 16q + 8h + i), real (part 0: A1, Z column 2kx) or imaginary (part 1: A2,
  // Z column 2kx + 1) contributions
  const int rt = w & 1, q = (w >> 1) & 1, part = w >> 2;
  const int zcol = l32 < m ? 2 * l32 + part : 0;  // columns kx >= m are not kept
  const int ar = rt * 32 + l32;
  const bool a_ok = ar < r4;
  f32x16_t acc = {};
  auto work = [&](const u32x4_t(&rv)[NU], const u32x4_t& av) {
    __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
    for (int u = 0; u < nu; ++u) *reinterpret_cast<u32x4_t*>(tile + prow[u] * ld + pcol[u]) = rv[u];
    if (has_a) *reinterpret_cast<u32x4_t*>(aslc + (a_part * r4 + a_row) * 40 + a_col) = av;
    __syncthreads();
    // x transform over this wave's 64-column slices
    f32x16_t z = {};
    for (int cs = w; cs < W / 64; cs += kSpecWaves) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 64 * cs + 16 * s + 8 * h;
        const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(tile + l32 * ld + k);
        bf16x8_t fb = *reinterpret_cast<const bf16x8_t*>(basis + (l32 < m2 ? l32 : 0) * ld + k);
        if (l32 >= m2) fb = bf16x8_t{};
        z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, fb, z, 0, 0, 0);
      }
    }
    __syncthreads();  // every wave has read the tile: its bytes now hold the parts of Z
    // this wave's part of Z: column j = l32 (< 2m), rows 8i + 4h .. 8i + 4h + 3
    if (l32 < m2) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const f32x4_t zz = {z[4 * i], z[4 * i + 1], z[4 * i + 2], z[4 * i + 3]};
        *reinterpret_cast<f32x4_t*>(zred + (w * m2 + l32) * kSpecZp + 8 * i + 4 * h) = zz;
      }
    }
    __syncthreads();
    // the y-transform product: Z column zcol, tile rows 16q + 8h .. + 7, summed over the
    // parts in wave order and rounded to BF16; A rows ar, the same tile rows
    f32x4_t lo = {}, hi = {};
#pragma unroll 2
    for (int ww = 0; ww < kSpecWaves; ++ww) {
      const float* zp = zred + (ww * m2 + zcol) * kSpecZp + 16 * q + 8 * h;
      lo += *reinterpret_cast<const f32x4_t*>(zp);
      hi += *reinterpret_cast<const f32x4_t*>(zp + 4);
    }
    uint16_t e[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      e[i] = f32_to_bf16(lo[i]);
      e[4 + i] = f32_to_bf16(hi[i]);
    }
    bf16x8_t af = bf16x8_t{};
    if (a_ok) af = *reinterpret_cast<const bf16x8_t*>(aslc + (part * r4 + ar) * 40 + 16 * q + 8 * h);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, __builtin_bit_cast(bf16x8_t, e), acc, 0, 0, 0);
  };
  // tiles in flight: the one being worked on and the next, in fixed registers. Every
  // trip issues the same loads (past the last tile, the last one again), so the waits
  // before a tile's LDS writes leave the next tile's loads in flight.
  u32x4_t r0[NU], r1[NU], q0, q1;
  load(r0, q0, 0);
#pragma unroll
  for (int i = 0; i < kBasisPieces; ++i) {
    const int idx = t + i * kThreads;
    if (idx < nbp) *reinterpret_cast<u32x4_t*>(basis + (idx / segs) * ld + (idx % segs) * 8) = bv[i];
  }
  for (int tl = 0; tl < tiles; tl += 2) {
    load(r1, q1, tl + 1 < tiles ? tl + 1 : tiles - 1);
    work(r0, q0);
    if (tl + 1 >= tiles) break;
    load(r0, q0, tl + 2 < tiles ? tl + 2 : tiles - 1);
    work(r1, q1);
  }
  // T = the sum of the waves' parts, in wave order: wave w holds rows 32 (w % 2) + 8i +
  // 4h + j, column kx = l32
  __syncthreads();
  float* red = reinterpret_cast<float*>(spec_smem);  // [wave][32][16]
  if (l32 < 16) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) red[(w * 32 + 8 * i + 4 * h + j) * 16 + l32] = acc[4 * i + j];
  }
  __syncthreads();
  // per plane, [plane][r][kx]; or mode-major, [r][kx][plane] (the backward's dS)
  for (int idx = t; idx < r4 * m; idx += kThreads) {
    const int r = idx / m, kx = idx % m, hr = r >> 5, rr = r & 31;
    float sum = 0.f;
#pragma unroll
    for (int ww = 0; ww < kSpecWaves; ww += 2) sum += red[((ww + hr) * 32 + rr) * 16 + kx];
    if constexpr (kModeMajor) {
      T[static_cast<long long>(idx) * gridDim.x + blockIdx.x] = sum;
    } else {
      T[static_cast<long long>(blockIdx.x) * r4 * m + idx] = sum;
    }
  }
}

// mode_major: T stored [r][kx][plane] instead of [plane][r][kx]
hipError_t launch_spectral_in(const uint16_t* v, long long sample_stride, long long plane_stride,
                              int planes_per_sample, int planes, const uint16_t* fxt,
                              const uint16_t* a1, const uint16_t* a2, int H, int W, int m,
                              float* T, hipStream_t stream, bool mode_major = false) {
  using Kernel = void (*)(const uint16_t*, long long, long long, int, const uint16_t*,
                          const uint16_t*, const uint16_t*, int, int, int, float*);
  static const Kernel table[2][4] = {
      {spectral_in_kernel<1, false>, spectral_in_kernel<2, false>, spectral_in_kernel<3, false>,
       spectral_in_kernel<4, false>},
      {spectral_in_kernel<1, true>, spectral_in_kernel<2, true>, spectral_in_kernel<3, true>,
       spectral_in_kernel<4, true>}};
  hipLaunchKernelGGL(table[mode_major][W / 128 - 1], dim3(static_cast<unsigned>(planes)),
                     dim3(64 * kSpecWaves), spectral_in_lds(W, m), stream, v, sample_stride,
                     plane_stride, planes_per_sample, fxt, a1, a2, H, W, m, T);
  return hipGetLastError();
}

// The inverse y transform of the kept modes, and the matching backward product:
//   U[plane][y][2kx + p] = sum_{k < 4m} Yp[y][k] S[plane][k][kx]   (p = 0: Ya, 1: Yb),
// forward with (Ya, Yb) = (IY1, IY2), S the mixed spectrum; backward with the transposed y
// bases (A1^T, A2^T) and S = dT, giving dZ. One block per plane: each of its 4 waves reads
// the plane's S (4m x m BF16) into the B operands of 32 x 32 x 16 products (lane kx, k
// slots 8h .. 8h + 7 of each 16-mode step), then for its 32-row tiles of y (w, w + 4, ...)
// the rows of Ya and Yb are the A operands (read from L2, the next tile's in flight) and
// the two accumulators give U's real and imaginary columns, written as (re, im) pairs.
// The two strided GEMMs this replaces ran 64 x 64 tiles for a 32 x 12 result per tile.
constexpr int kOutMaxM = 16;  // 4m <= 64 modes: at most 4 steps of 16

bool spectral_out_fits(int m) { return m >= 1 && m <= kOutMaxM; }

__device__ __forceinline__ bf16x8_t y_fragment(const uint16_t* __restrict__ Y, int y, int H,
                                               int k0, int r4) {
  // Y[y][k0 .. k0 + 7] (rows of 4m BF16: 8-byte aligned halves, each wholly in or out)
  uint2 lo = {0u, 0u}, hi = {0u, 0u};
  if (y < H) {
    const uint16_t* row = Y + static_cast<long long>(y) * r4 + k0;
    if (k0 < r4) lo = *reinterpret_cast<const uint2*>(row);
    if (k0 + 4 < r4) hi = *reinterpret_cast<const uint2*>(row + 4);
  }
  return __builtin_bit_cast(bf16x8_t, uint4{lo.x, lo.y, hi.x, hi.y});
}

__global__ __launch_bounds__(256) void spectral_out_kernel(
    const uint16_t* __restrict__ S, const uint16_t* __restrict__ Ya,
    const uint16_t* __restrict__ Yb, int H, int m, uint16_t* __restrict__ U) {
  const int lane = threadIdx.x & 63, l32 = lane & 31, h = lane >> 5;
  const int plane = blockIdx.x, w = threadIdx.x >> 6;  // wave w: row tiles w, w + 4, ...
  const int r4 = 4 * m, steps = (r4 + 15) / 16;
  // B operands: S[16s + 8h + i][kx = l32] (zero beyond the kept modes)
  const uint16_t* Sp = S + static_cast<long long>(plane) * r4 * m;
  bf16x8_t sb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    uint16_t e[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = 16 * s + 8 * h + i;
      e[i] = (s < steps && k < r4 && l32 < m) ? Sp[k * m + l32] : uint16_t(0);
    }
    sb[s] = __builtin_bit_cast(bf16x8_t, e);
  }
  uint16_t* Up = U + static_cast<long long>(plane) * H * 2 * m;
  const int tiles = (H + 31) / 32;
  bf16x8_t fa[4], fb[4], na[4], nb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    fa[s] = y_fragment(Ya, 32 * w + l32, H, 16 * s + 8 * h, r4);
    fb[s] = y_fragment(Yb, 32 * w + l32, H, 16 * s + 8 * h, r4);
  }
  for (int tl = w; tl < tiles; tl += 4) {
    const int y0 = tl * 32;
    if (tl + 4 < tiles) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        na[s] = y_fragment(Ya, y0 + 128 + l32, H, 16 * s + 8 * h, r4);
        nb[s] = y_fragment(Yb, y0 + 128 + l32, H, 16 * s + 8 * h, r4);
      }
    }
    f32x16_t re = {}, im = {};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s < steps) {
        re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], sb[s], re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fb[s], sb[s], im, 0, 0, 0);
      }
    }
    // lane kx holds rows y0 + 8i + 4h + j of columns 2kx (re) and 2kx + 1 (im)
    if (l32 < m) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int y = y0 + 8 * i + 4 * h + j;
          if (y < H) {
            const unsigned pair = static_cast<unsigned>(f32_to_bf16(re[4 * i + j])) |
                                  static_cast<unsigned>(f32_to_bf16(im[4 * i + j])) << 16;
            *reinterpret_cast<unsigned*>(Up + (static_cast<long long>(y) * m + l32) * 2) = pair;
          }
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      fa[s] = na[s];
      fb[s] = nb[s];
    }
  }
}

// The backward of the inverse y transform, into the mode-major dS:
//   dS[r][kx][plane] = sum_y YaT[r][y] Z[plane][y][2kx] + YbT[r][y] Z[plane][y][2kx + 1]
// (YaT, YbT: the transposed inverse y bases IY1^T, IY2^T, [4m][H]; Z = dU, [plane][H][2m]).
// One block per plane; each of its 4 waves takes 32-row tiles of y (w, w + 4, ...): the tile
// (32 rows of 2m BF16, contiguous) is loaded with 16-byte loads and stored transposed into the
// wave's LDS tile, whose rows (one per column j of Z) are the B operands of 32 x 32 x 16
// products; the rows of YaT and YbT are the A operands. The waves' accumulators (two 32-row
// tiles of T's 4m rows) are summed in a fixed order at the end.
__global__ __launch_bounds__(256) void spectral_y_kernel(
    const uint16_t* __restrict__ Z, const uint16_t* __restrict__ YaT,
    const uint16_t* __restrict__ YbT, int H, int m, float* __restrict__ dS) {
  __shared__ __attribute__((aligned(16))) uint16_t zt[4][32][40];  // [wave][column j][row]
  __shared__ float red[4][64][17];
  const int lane = threadIdx.x & 63, l32 = lane & 31, h = lane >> 5, w = threadIdx.x >> 6;
  const int plane = blockIdx.x, planes = gridDim.x;
  const int m2 = 2 * m, r4 = 4 * m, tiles = (H + 31) / 32;
  const uint16_t* Zp = Z + static_cast<long long>(plane) * H * m2;
  const bool vec = (H * m2) % 8 == 0;
  f32x16_t acc[2] = {};
  for (int tl = w; tl < tiles; tl += 4) {
    const int y0 = tl * 32, rows = min(32, H - y0), n = rows * m2;
    const uint16_t* src = Zp + static_cast<long long>(y0) * m2;
    // the tile, transposed into zt[j][y - y0] (rows beyond H and columns beyond 2m are zero)
    for (int i = lane; i < 32 * 32; i += 64) zt[w][i >> 5][i & 31] = 0;
    __builtin_amdgcn_wave_barrier();
    if (vec) {  // 16-byte pieces (H 2m a multiple of 8: every piece aligned and whole)
      for (int cidx = lane; cidx < n / 8; cidx += 64) {
        const u32x4_t q = *reinterpret_cast<const u32x4_t*>(src + 8 * cidx);
        uint16_t e[8];
        __builtin_memcpy(e, &q, 16);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int el = 8 * cidx + i;
          zt[w][el % m2][el / m2] = e[i];
        }
      }
    } else {
      for (int el = lane; el < n; el += 64) zt[w][el % m2][el / m2] = src[el];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int s = 0; s < 2; ++s) {  // tile rows 16 s + 8 h .. + 7 in the k slots of lane half h
      const int ks = 16 * s + 8 * h;
      const bf16x8_t bre = *reinterpret_cast<const bf16x8_t*>(&zt[w][(2 * l32) & 31][ks]);
      const bf16x8_t bim = *reinterpret_cast<const bf16x8_t*>(&zt[w][(2 * l32 + 1) & 31][ks]);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int r = rt * 32 + l32, y = y0 + ks;
        bf16x8_t fa = bf16x8_t{}, fb = bf16x8_t{};
        if (r < r4 && y + 8 <= H && H % 8 == 0) {  // rows of the bases 16-byte aligned
          fa = *reinterpret_cast<const bf16x8_t*>(YaT + static_cast<long long>(r) * H + y);
          fb = *reinterpret_cast<const bf16x8_t*>(YbT + static_cast<long long>(r) * H + y);
        } else if (r < r4) {
          uint16_t ea[8], eb[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            ea[i] = y + i < H ? YaT[static_cast<long long>(r) * H + y + i] : uint16_t(0);
            eb[i] = y + i < H ? YbT[static_cast<long long>(r) * H + y + i] : uint16_t(0);
          }
          fa = __builtin_bit_cast(bf16x8_t, ea);
          fb = __builtin_bit_cast(bf16x8_t, eb);
        }
        acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, bre, acc[rt], 0, 0, 0);
        acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fb, bim, acc[rt], 0, 0, 0);
      }
    }
    __builtin_amdgcn_wave_barrier();  // the tile is read before the next one is stored
  }
  // lane kx (< m) holds rows rt 32 + 8i + 4h + jj of column kx; sum the waves in order
  if (l32 < 16) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) red[w][rt * 32 + 8 * i + 4 * h + jj][l32] = acc[rt][4 * i + jj];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < r4 * m; idx += 256) {
    const int r = idx / m, kx = idx % m;
    dS[static_cast<long long>(idx) * planes + plane] =
        red[0][r][kx] + red[1][r][kx] + red[2][r][kx] + red[3][r][kx];
  }
}

hipError_t launch_spectral_y(const uint16_t* Z, const uint16_t* YaT, const uint16_t* YbT,
                             int planes, int H, int m, float* dS, hipStream_t stream) {
  hipLaunchKernelGGL(spectral_y_kernel, dim3(static_cast<unsigned>(planes)), dim3(256), 0,
                     stream, Z, YaT, YbT, H, m, dS);
  return hipGetLastError();
}

hipError_t launch_spectral_out(const uint16_t* S, const uint16_t* Ya, const uint16_t* Yb,
                               int planes, int H, int m, uint16_t* U, hipStream_t stream) {
  hipLaunchKernelGGL(spectral_out_kernel, dim3(static_cast<unsigned>(planes)), dim3(256), 0,
                     stream, S, Ya, Yb, H, m, U);
  return hipGetLastError();
}

// Mode mixing of a Fourier layer and its two backward products. The spectra T, S and dT are
// stored per plane, [(b, c)][2 kyi + p][kx] (p = 0: real part, 1: imaginary part); dS, which
// only the backward mixing reads, is stored mode-major, [2 kyi + p][kx][(b, o)], so that one
// mode's values of every (b, o) are contiguous (storing T that way as well made the one-pass
// transform that writes it slower by more than the mixing gained). R is [mode][c][o][2] with
// mode = kyi m + kx. Blocks (mode, q), q < kModeSplit: the mode's spectral values of every
// (b, c) are read into LDS, the block's part of R's C x C block of the mode is read
// contiguously, and the products run out of LDS (sample b in chunks of kModeRows / C); block
// q computes the q-th quarter of the output channels (of the rows c of dR). One block per mode
// (288 at 12 modes) left most of the chip idle.
// The complex products are written as real pairs:
//   S    = sum_c R[c][o] T[c]:       (rr tr - ri ti, rr ti + ri tr)
//   dT   = sum_o conj(R[c][o]) dS[o]: (rr dr + ri di, rr di - ri dr)
//   dR  += sum_b conj(T[b][c]) dS[b][o]: (tr dr + ti di, tr di - ti dr)
constexpr int kModeC = 64;        // channel limit of the per-mode kernels
constexpr int kModeRows = 1024;   // (b, c) pairs staged per chunk
constexpr int kModeSplit = 4;     // blocks per mode, each a quarter of the output channels

__device__ __forceinline__ size_t spec_at(int b, int c, int C, int m, int kyi, int kx) {
  return (static_cast<size_t>(b) * C + c) * (4 * m * m) + static_cast<size_t>(2 * kyi) * m + kx;
}
// The mode-major spectrum dS ([2kyi + p][kx][plane] over planes (b, o)): the real parts of
// mode (kyi, kx) start here, the imaginary parts m * planes further on.
__device__ __forceinline__ size_t mode_base(int m, int kyi, int kx, size_t planes) {
  return (static_cast<size_t>(2 * kyi) * m + kx) * planes;
}

// S[(b,o)] at one mode = sum_c R[mode][c][o] T[(b,c)] (complex), stored BF16.
__global__ __launch_bounds__(256) void mix_forward_kernel(const float* __restrict__ T,
                                                          const float* __restrict__ R,
                                                          uint16_t* __restrict__ S, int B, int C,
                                                          int m) {
  __shared__ float rs[kModeC * kModeC * 2];  // R[c][o][2] of this mode, this block's o
  __shared__ float tre[kModeRows], tim[kModeRows];
  const int mode = blockIdx.x, kyi = mode / m, kx = mode % m, t = threadIdx.x;
  const int osz = (C + kModeSplit - 1) / kModeSplit, o0 = blockIdx.y * osz;
  const int no = min(C, o0 + osz) - o0;  // this block's output channels o0 .. o0 + no - 1
  if (no <= 0) return;
  const float* rm = R + static_cast<size_t>(mode) * C * C * 2;
  for (int i = t; i < C * no; i += 256) {
    const int c = i / no, ol = i % no;
    rs[(c * no + ol) * 2] = rm[(c * C + o0 + ol) * 2];
    rs[(c * no + ol) * 2 + 1] = rm[(c * C + o0 + ol) * 2 + 1];
  }
  const int per = kModeRows / C;  // samples per chunk
  for (int b0 = 0; b0 < B; b0 += per) {
    const int nb = min(per, B - b0);
    __syncthreads();
    for (int i = t; i < nb * C; i += 256) {
      const size_t at = spec_at(b0 + i / C, i % C, C, m, kyi, kx);
      tre[i] = T[at];
      tim[i] = T[at + m];
    }
    __syncthreads();
    for (int i = t; i < nb * no; i += 256) {  // output (b, o): consecutive threads, consecutive o
      const int bl = i / no, ol = i % no, o = o0 + ol;
      float sr = 0.f, si = 0.f;
      for (int c = 0; c < C; ++c) {
        const float rr = rs[(c * no + ol) * 2], ri = rs[(c * no + ol) * 2 + 1];
        const float tr = tre[bl * C + c], ti = tim[bl * C + c];
        sr = fmaf(rr, tr, fmaf(-ri, ti, sr));
        si = fmaf(rr, ti, fmaf(ri, tr, si));
      }
      const size_t at = spec_at(b0 + bl, o, C, m, kyi, kx);
      S[at] = f32_to_bf16(sr);
      S[at + m] = f32_to_bf16(si);
    }
  }
}

// dT[(b,c)] at one mode = sum_o conj(R[mode][c][o]) dS[(b,o)], stored BF16.
__global__ __launch_bounds__(256) void mix_backward_input_kernel(const float* __restrict__ dS,
                                                                 const float* __restrict__ R,
                                                                 uint16_t* __restrict__ dT,
                                                                 int B, int C, int m) {
  __shared__ float rs[kModeC * kModeC * 2];  // R[o][c][2] of this mode (transposed), this block's c
  __shared__ float dre[kModeRows], dim_[kModeRows];
  const int mode = blockIdx.x, kyi = mode / m, kx = mode % m, t = threadIdx.x;
  const int csz = (C + kModeSplit - 1) / kModeSplit, c0 = blockIdx.y * csz;
  const int nc = min(C, c0 + csz) - c0;  // this block's output channels c0 .. c0 + nc - 1
  if (nc <= 0) return;
  const float* rm = R + static_cast<size_t>(mode) * C * C * 2;
  for (int i = t; i < nc * C; i += 256) {  // i = cl C + o: R's rows c, read contiguously
    const int cl = i / C, o = i % C;
    rs[(o * nc + cl) * 2] = rm[((c0 + cl) * C + o) * 2];
    rs[(o * nc + cl) * 2 + 1] = rm[((c0 + cl) * C + o) * 2 + 1];
  }
  const size_t planes = static_cast<size_t>(B) * C, db = mode_base(m, kyi, kx, planes);
  const size_t mp = static_cast<size_t>(m) * planes;
  const int per = kModeRows / C;
  for (int b0 = 0; b0 < B; b0 += per) {
    const int nb = min(per, B - b0);
    __syncthreads();
    for (int i = t; i < nb * C; i += 256) {  // planes b0 C + i, contiguous
      dre[i] = dS[db + static_cast<size_t>(b0) * C + i];
      dim_[i] = dS[db + mp + static_cast<size_t>(b0) * C + i];
    }
    __syncthreads();
    for (int i = t; i < nb * nc; i += 256) {  // output (b, c): consecutive threads, consecutive c
      const int bl = i / nc, cl = i % nc, c = c0 + cl;
      float gr = 0.f, gi = 0.f;
      for (int o = 0; o < C; ++o) {
        const float rr = rs[(o * nc + cl) * 2], ri = rs[(o * nc + cl) * 2 + 1];
        const float dr = dre[bl * C + o], di = dim_[bl * C + o];
        gr = fmaf(rr, dr, fmaf(ri, di, gr));
        gi = fmaf(rr, di, fmaf(-ri, dr, gi));
      }
      const size_t at = spec_at(b0 + bl, c, C, m, kyi, kx);
      dT[at] = f32_to_bf16(gr);
      dT[at + m] = f32_to_bf16(gi);
    }
  }
}

// dR[mode][c][o] += sum_b conj(T[(b,c)]) dS[(b,o)] at one mode.
__global__ __launch_bounds__(256) void mix_backward_weight_kernel(const float* __restrict__ dS,
                                                                  const float* __restrict__ T,
                                                                  float* __restrict__ dR, int B,
                                                                  int C, int m) {
  __shared__ float tre[kModeRows], tim[kModeRows], dre[kModeRows], dim_[kModeRows];
  constexpr int kOut = (kModeC * kModeC / kModeSplit + 255) / 256;  // outputs per thread
  const int mode = blockIdx.x, kyi = mode / m, kx = mode % m, t = threadIdx.x;
  const int csz = (C + kModeSplit - 1) / kModeSplit, c0 = blockIdx.y * csz;
  const int nc = min(C, c0 + csz) - c0;  // this block's rows c0 .. c0 + nc - 1 of dR
  if (nc <= 0) return;
  float ar[kOut], ai[kOut];
#pragma unroll
  for (int k = 0; k < kOut; ++k) ar[k] = ai[k] = 0.f;
  const size_t planes = static_cast<size_t>(B) * C, base = mode_base(m, kyi, kx, planes);
  const size_t mp = static_cast<size_t>(m) * planes;
  const int per = kModeRows / C;
  for (int b0 = 0; b0 < B; b0 += per) {
    const int nb = min(per, B - b0);
    __syncthreads();
    for (int i = t; i < nb * C; i += 256) {
      const size_t at = spec_at(b0 + i / C, i % C, C, m, kyi, kx);  // T: per plane
      tre[i] = T[at];
      tim[i] = T[at + m];
      const size_t ad = base + static_cast<size_t>(b0) * C + i;      // dS: planes contiguous
      dre[i] = dS[ad];
      dim_[i] = dS[ad + mp];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kOut; ++k) {  // output j = cl C + o: consecutive threads, consecutive o
      const int j = t + 256 * k;
      if (j >= nc * C) break;
      const int c = c0 + j / C, o = j % C;
      for (int bl = 0; bl < nb; ++bl) {
        const float tr = tre[bl * C + c], ti = tim[bl * C + c];
        const float dr = dre[bl * C + o], di = dim_[bl * C + o];
        ar[k] = fmaf(tr, dr, fmaf(ti, di, ar[k]));
        ai[k] = fmaf(tr, di, fmaf(-ti, dr, ai[k]));
      }
    }
  }
  float* rm = dR + (static_cast<size_t>(mode) * C + c0) * C * 2;  // rows c0 ..
#pragma unroll
  for (int k = 0; k < kOut; ++k) {
    const int j = t + 256 * k;
    if (j >= nc * C) break;
    rm[2 * j] += ar[k];
    rm[2 * j + 1] += ai[k];
  }
}

// Weight and bias gradients of a pointwise (1x1) layer on the matrix cores, for Mo <= 32 MH
// output and K <= 32 NH input channels: dW[mo][k] += sum_{b,p} d[b][mo][p] x[b][k][p] and
// db[mo] += sum_{b,p} d[b][mo][p]. A block takes a contiguous run of steps of PX pixels of one
// sample. In a step its waves copy the step's slice of every row of d and x to LDS with
// direct-to-LDS loads, each load one contiguous 1 KB (two rows of 512 bytes, or four of 256),
// then every wave multiplies an eighth of the slice on the MFMAs, reading its fragments
// (lane l: row l % 32, 8 pixels) from LDS. The 16-byte chunk c of staged row r sits in slot
// c ^ (r % 16), so the 16 rows that one LDS read phase touches fall in distinct banks. Rows
// past Mo or K are not loaded (or load the last row) and only reach outputs that are never
// stored; pixels past the end of a sample (P a multiple of 64, not of PX) are zeroed. The bias
// gradient adds the d fragments by dot products with ones. The waves of a block add their
// sums in LDS in a fixed order into one partial per block, and wgrad_final_kernel adds the
// partials of all blocks in a fixed order: the result does not depend on scheduling.
// Eight waves per block measured 1% faster in training than four (2098 against 2080 samples/s
// at 512^2, batch 16); 128-pixel steps for every shape on top of that, 1% slower.
constexpr int kWgWaves = 8, kWgPix = 64, kWgBlocks = 1024;
constexpr int kWgMaxE = 8 * 1024 + 4 * 64;  // floats of one partial at MH NH = 8, MH = 4

// 16 bytes per lane from global memory straight into LDS: lane i's bytes land at lds + 16 i
// (lds wave-uniform). The builtin is kept out of the host pass, where it would drop the
// host-side launch stubs of the kernel templates that use it.
__device__ __forceinline__ void load_to_lds16(const void* src, void* lds) {
#if __HIP_DEVICE_COMPILE__
  __builtin_amdgcn_global_load_lds(src, lds, 16, 0, 0);
#else
  (void)src;
  (void)lds;
#endif
}

template <int MH, int NH>
struct WgShape {
  static constexpr int kRows = 32 * (MH + NH);                 // staged rows: d, then x
  static constexpr int kPx = kRows <= 128 ? 256 : 128;          // pixels per step
  static constexpr int kRowBytes = 2 * kPx;
  static constexpr int kLds = kRows * kRowBytes;
  static constexpr int kE = MH * NH * 1024 + MH * 64;          // floats of one partial
};

template <int MH, int NH>
__global__ __launch_bounds__(64 * kWgWaves, 2) void wgrad_kernel(
    const uint16_t* __restrict__ d, int Mo, const uint16_t* __restrict__ x, int K, long long P,
    long long steps, float* __restrict__ part) {
  using S = WgShape<MH, NH>;
  constexpr int kT = MH * NH, kE = S::kE, kPx = S::kPx, kRB = S::kRowBytes;
  constexpr int kChunks = kPx / 8;                 // 16-byte chunks of a staged row
  constexpr int kRowsPerLoad = 64 / kChunks;       // rows one wave load fills (2 or 4)
  constexpr int kLoads = S::kRows / kRowsPerLoad;  // wave loads per step
  constexpr int kSub = kPx / (16 * kWgWaves);      // MFMA k steps per wave per step
  static_assert(S::kLds >= kE * 4, "the partial fits the staging buffer");
  static_assert(kSub >= 1 && kSub * 16 * kWgWaves == kPx, "the waves split a step evenly");
  __shared__ __attribute__((aligned(16))) unsigned char lds[S::kLds];
  const int lane = threadIdx.x & 63, r = lane & 31, hf = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long spp = (P + kPx - 1) / kPx;  // steps per sample
  long long s = steps * blockIdx.x / gridDim.x;
  const long long s1 = steps * (blockIdx.x + 1) / gridDim.x;
  long long b = s / spp, p0 = (s - b * spp) * kPx;
  const int lr = lane / kChunks, slot = lane % kChunks;  // this lane's row and slot in a load
  f32x16_t acc[MH][NH];
  float dsum[MH];
#pragma unroll
  for (int i = 0; i < MH; ++i) {
    dsum[i] = 0.f;
#pragma unroll
    for (int j = 0; j < NH; ++j) acc[i][j] = f32x16_t{};
  }
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  const bf16x2_t ones = {static_cast<__bf16>(1.f), static_cast<__bf16>(1.f)};
  for (; s < s1; ++s) {
    for (int q = wave; q < kLoads; q += kWgWaves) {
      const int row0 = q * kRowsPerLoad, row = row0 + lr;  // staged rows of this load
      const bool is_d = row0 < 32 * MH;
      const int first = is_d ? row0 : row0 - 32 * MH, n = is_d ? Mo : K;
      if (first >= n) continue;  // every row of this load is past the last one
      const int c = slot ^ (row & 15);
      const long long pc = p0 + 8 * c, px = pc < P - 8 ? pc : P - 8;
      const uint16_t* src = is_d ? d + (b * Mo + min(row, Mo - 1)) * P + px
                                 : x + (b * K + min(row - 32 * MH, K - 1)) * P + px;
      load_to_lds16(src, lds + row0 * kRB);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kSub; ++t) {
      const int pl = (wave * kSub + t) * 16 + 8 * hf;  // this lane's 8 pixels in the step
      const bool ok = p0 + pl < P;
      const int c = pl / 8;
      u32x4_t fb[NH];
#pragma unroll
      for (int j = 0; j < NH; ++j) {
        const int row = 32 * MH + 32 * j + r;
        fb[j] = *reinterpret_cast<const u32x4_t*>(lds + row * kRB + ((c ^ (row & 15)) << 4));
        if (!ok) fb[j] = u32x4_t{};
      }
#pragma unroll
      for (int i = 0; i < MH; ++i) {
        const int row = 32 * i + r;
        u32x4_t fa = *reinterpret_cast<const u32x4_t*>(lds + row * kRB + ((c ^ (row & 15)) << 4));
        if (!ok) fa = u32x4_t{};
        const bf16x8_t av = __builtin_bit_cast(bf16x8_t, fa);
#pragma unroll
        for (int j = 0; j < NH; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              av, __builtin_bit_cast(bf16x8_t, fb[j]), acc[i][j], 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          // a copy: __builtin_bit_cast of a vector element in place reads element 0
          const unsigned w = fa[e];
          dsum[i] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w), ones,
                                                    dsum[i], false);
        }
      }
    }
    __syncthreads();
    p0 += kPx;
    if (p0 >= P) {
      p0 = 0;
      ++b;
    }
  }
  // waves 7, 6, ..., 1 pass their running sum down through LDS; wave 0 stores the block's
  // (separate LDS and global stores: one pointer that may be either costs flat addresses)
  float* red = reinterpret_cast<float*>(lds);
  auto to_lds = [&](bool add) {
#pragma unroll
    for (int i = 0; i < MH; ++i) {
#pragma unroll
      for (int j = 0; j < NH; ++j)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = ((i * NH + j) * 16 + q) * 64 + lane;
          red[e] = add ? acc[i][j][q] + red[e] : acc[i][j][q];
        }
      const int e = kT * 1024 + i * 64 + lane;
      red[e] = add ? dsum[i] + red[e] : dsum[i];
    }
  };
  __syncthreads();
  if (wave == kWgWaves - 1) to_lds(false);
  for (int w = kWgWaves - 2; w >= 1; --w) {
    __syncthreads();
    if (wave == w) to_lds(true);
  }
  __syncthreads();
  if (wave == 0) {
    float* mine = part + static_cast<size_t>(blockIdx.x) * kE;
#pragma unroll
    for (int i = 0; i < MH; ++i) {
#pragma unroll
      for (int j = 0; j < NH; ++j)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = ((i * NH + j) * 16 + q) * 64 + lane;
          mine[e] = acc[i][j][q] + red[e];
        }
      const int e = kT * 1024 + i * 64 + lane;
      mine[e] = dsum[i] + red[e];
    }
  }
}

// dW[mo][k] += and db[mo] += the sums over the nblk partials of wgrad_kernel. Output element
// f is a tile accumulator element (f < 1024 MH NH: register (f / 64) % 16 of lane f % 64 of
// tile f / 1024) or a bias row (both pixel halves of lanes r and r + 32). A block takes 16
// elements; its 64 groups of 16 threads each add every 64th partial, and the 64 sums are
// then added in order.
template <int MH, int NH>
__global__ __launch_bounds__(1024) void wgrad_final_kernel(const float* __restrict__ part,
                                                           int nblk, int Mo, int K,
                                                           float* __restrict__ dW,
                                                           float* __restrict__ db) {
  constexpr int kT = MH * NH, kE = WgShape<MH, NH>::kE, kF = kT * 1024 + MH * 32;
  __shared__ double tot[64][17];
  const int el = threadIdx.x & 15, sub = threadIdx.x >> 4;
  const int f = blockIdx.x * 16 + el;
  const bool tile = f < kT * 1024;
  int e0 = f, e1 = -1;  // the partial elements that make up f
  if (!tile) {
    const int g = f - kT * 1024;
    e0 = kT * 1024 + (g / 32) * 64 + g % 32;
    e1 = e0 + 32;
  }
  double acc = 0.0;
  if (f < kF) {
#pragma unroll 4
    for (int j = sub; j < nblk; j += 64) {
      const float* pj = part + static_cast<size_t>(j) * kE;
      acc += e1 < 0 ? static_cast<double>(pj[e0])
                    : static_cast<double>(pj[e0]) + static_cast<double>(pj[e1]);
    }
  }
  tot[sub][el] = acc;
  __syncthreads();
  if (sub != 0 || f >= kF) return;
  double v = 0.0;
  for (int q = 0; q < 64; ++q) v += tot[q][el];
  if (tile) {
    const int t = f / 1024, q = (f / 64) % 16, lane = f % 64, tm = t / NH, tn = t % NH;
    const int mo = 32 * tm + 8 * (q / 4) + 4 * (lane / 32) + q % 4, k = 32 * tn + lane % 32;
    if (mo < Mo && k < K) dW[static_cast<size_t>(mo) * K + k] += static_cast<float>(v);
  } else if (db) {
    const int mo = f - kT * 1024;
    if (mo < Mo) db[mo] += static_cast<float>(v);
  }
}

// The tile shape (MH, NH) of wgrad_kernel for Mo output and K input channels, or false.
bool wgrad_shape(int Mo, int K, long long P, int* mh, int* nh) {
  auto up = [](int n) { return n <= 32 ? 1 : n <= 64 ? 2 : n <= 128 ? 4 : 0; };
  const int a = up(Mo), c = up(K);
  if (Mo < 1 || K < 1 || !a || !c || a * c > 8 || P < kWgPix || P % kWgPix) return false;
  *mh = a;
  *nh = c;
  return true;
}

// One round of resident blocks (each then takes the same number of steps), at most what the
// partial buffer holds and at most one block per step.
template <int MH, int NH>
hipError_t launch_wgrad_t(const uint16_t* d, int Mo, const uint16_t* x, int K, int B, long long P,
                          int cus, float* part, float* dW, float* db, hipStream_t stream) {
  constexpr long long kE = WgShape<MH, NH>::kE, kPx = WgShape<MH, NH>::kPx;
  static const int occ = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wgrad_kernel<MH, NH>, 64 * kWgWaves,
                                                     0) != hipSuccess || n < 1)
      n = 1;
    return n;
  }();
  const long long steps = static_cast<long long>(B) * ((P + kPx - 1) / kPx);
  long long nb = std::min(steps, static_cast<long long>(occ) * std::max(cus, 1));
  nb = std::min(nb, static_cast<long long>(kWgBlocks) * kWgMaxE / kE);
  const int nblk = static_cast<int>(nb);
  hipLaunchKernelGGL((wgrad_kernel<MH, NH>), dim3(nblk), dim3(64 * kWgWaves), 0, stream, d, Mo,
                     x, K, P, steps, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((wgrad_final_kernel<MH, NH>), dim3((MH * NH * 1024 + MH * 32 + 15) / 16),
                     dim3(1024), 0, stream, part, nblk, Mo, K, dW, db);
  return hipGetLastError();
}

// dW (Mo x K, row-major) += d x^T and db += d 1 over every pixel of the batch, on a device
// with cus compute units; part holds kWgBlocks * kWgMaxE floats. The shape must pass
// wgrad_shape.
hipError_t launch_wgrad(const uint16_t* d, int Mo, const uint16_t* x, int K, int B, long long P,
                        int cus, float* part, float* dW, float* db, hipStream_t stream) {
  int mh = 0, nh = 0;
  if (B < 1 || !wgrad_shape(Mo, K, P, &mh, &nh)) return hipErrorInvalidValue;
  switch (mh * 8 + nh) {
    case 9: return launch_wgrad_t<1, 1>(d, Mo, x, K, B, P, cus, part, dW, db, stream);
    case 10: return launch_wgrad_t<1, 2>(d, Mo, x, K, B, P, cus, part, dW, db, stream);
    case 12: return launch_wgrad_t<1, 4>(d, Mo, x, K, B, P, cus, part, dW, db, stream);
    case 17: return launch_wgrad_t<2, 1>(d, Mo, x, K, B, P, cus, part, dW, db, stream);
    case 18: return launch_wgrad_t<2, 2>(d, Mo, x, K, B, P, cus, part, dW, db, stream);
    case 20: return launch_wgrad_t<2, 4>(d, Mo, x, K, B, P, cus, part, dW, db, stream);
    case 33: return launch_wgrad_t<4, 1>(d, Mo, x, K, B, P, cus, part, dW, db, stream);
    case 34: return launch_wgrad_t<4, 2>(d, Mo, x, K, B, P, cus, part, dW, db, stream);
    default: return hipErrorInvalidValue;
  }
}

// dz = dv * GELU'(z)
__global__ void gelu_grad_kernel(const float* __restrict__ dv, const uint16_t* __restrict__ z,
                                 uint16_t* __restrict__ dz, size_t n) {
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock)
    dz[i] = f32_to_bf16(dv[i] * gelu_prime_as(bf16_to_f32(z[i])));
}

// Block x of sample b writes part[2 (b X + x)] = its share of sum (out - target)^2 and
// part[2 (b X + x) + 1] = its share of sum target^2 (X = gridDim.x blocks per sample);
// loss_sums_kernel adds the shares in block order, so the sums repeat bit for bit.
constexpr int kLossBlocks = 256;
__global__ void loss_partial_kernel(const float* __restrict__ out, const uint16_t* __restrict__ tg,
                                    double* __restrict__ part, size_t per) {
  __shared__ double r0[kBlock], r1[kBlock];
  const int b = blockIdx.y;
  double a0 = 0.0, a1 = 0.0;
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < per; i += size_t(gridDim.x) * kBlock) {
    const double t = bf16_to_f32(tg[b * per + i]);
    const double d = out[b * per + i] - t;
    a0 += d * d;
    a1 += t * t;
  }
  r0[threadIdx.x] = a0;
  r1[threadIdx.x] = a1;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const size_t at = 2 * (static_cast<size_t>(b) * gridDim.x + blockIdx.x);
    part[at] = r0[0];
    part[at + 1] = r1[0];
  }
}

// sums[2b + k] = sum over the nblk shares part[2 (b nblk + x) + k] in order of x (one
// thread per sample and sum)
__global__ void loss_sums_kernel(const double* __restrict__ part, int nblk, int B,
                                 double* __restrict__ sums) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // 2 b + k
  if (i >= 2 * B) return;
  const int b = i / 2, k = i % 2;
  double acc = 0.0;
  for (int x = 0; x < nblk; ++x) acc += part[2 * (static_cast<size_t>(b) * nblk + x) + k];
  sums[i] = acc;
}

// loss = mean_b |out_b - t_b| / |t_b|;  dout = (out - t) / (B |out_b - t_b| |t_b|)
__global__ void loss_grad_kernel(const float* __restrict__ out, const uint16_t* __restrict__ tg,
                                 const double* __restrict__ sums, uint16_t* __restrict__ dout,
                                 int B, size_t per) {
  const int b = blockIdx.y;
  const double nd = sqrt(sums[2 * b]), nt = sqrt(sums[2 * b + 1]);
  const float scale = (nd > 0.0 && nt > 0.0) ? static_cast<float>(1.0 / (B * nd * nt)) : 0.f;
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < per; i += size_t(gridDim.x) * kBlock) {
    const float d = out[b * per + i] - bf16_to_f32(tg[b * per + i]);
    dout[b * per + i] = f32_to_bf16(d * scale);
  }
}

__global__ void loss_final_kernel(const double* __restrict__ sums, int B, float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  for (int b = 0; b < B; ++b) acc += sums[2 * b + 1] > 0.0 ? sqrt(sums[2 * b] / sums[2 * b + 1]) : 0.0;
  *loss = static_cast<float>(acc / B);
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m1, float* __restrict__ m2, size_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a * c1) / (sqrtf(v * c2) + eps);
  }
}

// Network input (n - n_shift, q2, q3, q4) and target (q2, q3, q4) as BF16 planes.
__global__ void pack_kernel(const double* __restrict__ q, const double* __restrict__ n, size_t P,
                            double n_shift, uint16_t* __restrict__ in4, uint16_t* __restrict__ t3) {
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < P; i += size_t(gridDim.x) * kBlock) {
    if (in4) {
      in4[i] = f32_to_bf16(static_cast<float>(n[i] - n_shift));
      for (int c = 0; c < 3; ++c) in4[(c + 1) * P + i] = f32_to_bf16(static_cast<float>(q[c * P + i]));
    }
    if (t3)
      for (int c = 0; c < 3; ++c) t3[c * P + i] = f32_to_bf16(static_cast<float>(q[c * P + i]));
  }
}

// Energy sum q^2 over the three output channels of each sample of an FP32 batch.
__global__ void energy_batch_kernel(const float* __restrict__ out, double* __restrict__ e,
                                    size_t per) {
  __shared__ double r[kBlock];
  const int b = blockIdx.y;
  double a = 0.0;
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < per; i += size_t(gridDim.x) * kBlock) {
    const double v = out[b * per + i];
    a += v * v;
  }
  r[threadIdx.x] = a;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) r[threadIdx.x] += r[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(&e[b], r[0]);
}

// Band sums of sample b (blockIdx.y): sums[2b] += sum over the kept modes of
// w(kx) |F(ky, kx)|^2, where T[(b,c)][2 kyi + p][kx] holds the re/im parts of the
// truncated DFT and w = 1 at kx = 0, 2 otherwise (for a real field the mode
// (-ky, -kx) has the same magnitude and is not among the stored ones);
// sums[2b + 1] += sum of the squares of the nch input planes at in + b in_stride.
__global__ void band_sums_kernel(const float* __restrict__ T, const uint16_t* __restrict__ in,
                                 long long in_stride, int nch, size_t P, int m,
                                 double* __restrict__ sums) {
  __shared__ double r0[kBlock], r1[kBlock];
  const int b = blockIdx.y;
  const size_t per_t = size_t(nch) * 4 * m * m;
  const size_t stride = size_t(gridDim.x) * kBlock;
  double kept = 0.0, total = 0.0;
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < per_t; i += stride) {
    const double v = T[b * per_t + i];
    kept += (i % m == 0 ? 1.0 : 2.0) * v * v;
  }
  const uint16_t* x = in + b * in_stride;
  for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < size_t(nch) * P; i += stride) {
    const double v = bf16_to_f32(x[i]);
    total += v * v;
  }
  r0[threadIdx.x] = kept;
  r1[threadIdx.x] = total;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&sums[2 * b], r0[0]);
    atomicAdd(&sums[2 * b + 1], r1[0]);
  }
}

// fraction[b] = kept / (H W total) (Parseval), 0 for a zero sample.
__global__ void band_final_kernel(const double* __restrict__ sums, int B, double hw,
                                  double* __restrict__ fraction) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) fraction[b] = sums[2 * b + 1] > 0.0 ? sums[2 * b] / (hw * sums[2 * b + 1]) : 0.0;
}

// Small deterministic generator for the initial weights (splitmix64).
struct Rng {
  uint64_t s;
  double uniform() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0);
  }
};

}  // namespace

struct qla_fno {
  int H = 0, W = 0, P = 0, Cin = 0, C = 0, C2 = 0, Cout = 0, L = 0, m = 0, Bmax = 0;
  int device = 0, cus = 1;  // device and its compute units
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // flat parameter layout
  size_t nparam = 0, o_Wp = 0, o_bp = 0, o_Q1 = 0, o_bq1 = 0, o_Q2 = 0, o_bq2 = 0;
  std::vector<size_t> o_W, o_b, o_R;
  size_t nweights16 = 0;  // BF16 copies: Wp | W_0..W_{L-1} | Q1 | Q2
  float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
  uint16_t* w16 = nullptr;
  uint16_t *Fx = nullptr, *FxT = nullptr, *A1 = nullptr, *A2 = nullptr, *A1T = nullptr,
           *A2T = nullptr, *IY1 = nullptr, *IY2 = nullptr, *IY1T = nullptr, *IY2T = nullptr,
           *IX = nullptr;
  // activations (batch Bmax)
  std::vector<uint16_t*> v, z;
  uint16_t *Zb = nullptr, *Sb = nullptr, *Ub = nullptr, *zq = nullptr, *h = nullptr,
           *dout = nullptr, *dzq = nullptr, *dza = nullptr, *dzb = nullptr, *dU = nullptr,
           *dT = nullptr, *dZ = nullptr;
  std::vector<float*> T;
  // spec and dv (FP32) only when W is not a multiple of the GEMM column tile, where
  // the inverse x transform cannot be fused into the channel-mixing GEMM
  float *spec = nullptr, *out = nullptr, *dS = nullptr, *dv = nullptr, *loss = nullptr;
  float* wpart = nullptr;  // per-block partial sums of the weight-gradient kernel
  bool fused = false;
  double* sums = nullptr;
  double* lpart = nullptr;  // per-block shares of the loss sums
  double* band = nullptr;  // per-sample band sums of qla_fno_band_fraction
  int64_t adam_t = 0;
  std::vector<void*> allocs;

  size_t w16_Wp() const { return 0; }
  size_t w16_W(int l) const { return size_t(C) * Cin + size_t(l) * C * C; }
  size_t w16_Q1() const { return size_t(C) * Cin + size_t(L) * C * C; }
  size_t w16_Q2() const { return w16_Q1() + size_t(C2) * C; }
};

namespace {

qla_status dalloc(qla_fno* f, void** p, size_t bytes) {
  const hipError_t e = hipMalloc(p, bytes ? bytes : 16);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(QLA_ENOMEM, std::string("FNO allocation: ") + hipGetErrorString(e));
  }
  f->allocs.push_back(*p);
  return QLA_OK;
}

template <typename P>
qla_status dalloc_t(qla_fno* f, P** p, size_t count) {
  return dalloc(f, reinterpret_cast<void**>(p), count * sizeof(P));
}

void release(qla_fno* f) {
  for (void* p : f->allocs) (void)hipFree(p);
  f->allocs.clear();
  if (f->own_stream && f->stream) (void)hipStreamDestroy(f->stream);
}

std::vector<uint16_t> to_bf16(const std::vector<double>& v) {
  std::vector<uint16_t> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = f32_to_bf16(static_cast<float>(v[i]));
  return o;
}

qla_status upload16(qla_fno* f, uint16_t** dst, const std::vector<double>& v) {
  qla_status st = dalloc_t(f, dst, v.size());
  if (st != QLA_OK) return st;
  const std::vector<uint16_t> h = to_bf16(v);
  QLA_HIP(hipMemcpy(*dst, h.data(), h.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  return QLA_OK;
}

// The cosine/sine bases of the truncated transforms (see the header comment).
qla_status make_bases(qla_fno* f) {
  const int H = f->H, W = f->W, m = f->m;
  const double two_pi = 6.283185307179586476925286766559;
  std::vector<double> Fx(size_t(W) * 2 * m), IX(size_t(2 * m) * W);
  for (int x = 0; x < W; ++x)
    for (int kx = 0; kx < m; ++kx) {
      const double a = two_pi * kx * x / W;
      Fx[size_t(x) * 2 * m + 2 * kx] = std::cos(a);
      Fx[size_t(x) * 2 * m + 2 * kx + 1] = -std::sin(a);
      const double w = (kx == 0 ? 1.0 : 2.0) / (double(H) * W);
      IX[size_t(2 * kx) * W + x] = w * std::cos(a);
      IX[size_t(2 * kx + 1) * W + x] = -w * std::sin(a);
    }
  std::vector<double> A1(size_t(4 * m) * H), A2(size_t(4 * m) * H), IY1(size_t(H) * 4 * m),
      IY2(size_t(H) * 4 * m);
  for (int kyi = 0; kyi < 2 * m; ++kyi) {
    const int ky = kyi < m ? kyi : H - 2 * m + kyi;
    for (int y = 0; y < H; ++y) {
      const double a = two_pi * double(ky) * y / H, c = std::cos(a), s = std::sin(a);
      A1[size_t(2 * kyi) * H + y] = c;       // T_re from Z_re
      A1[size_t(2 * kyi + 1) * H + y] = -s;  // T_im from Z_re
      A2[size_t(2 * kyi) * H + y] = s;       // T_re from Z_im
      A2[size_t(2 * kyi + 1) * H + y] = c;   // T_im from Z_im
      IY1[size_t(y) * 4 * m + 2 * kyi] = c;       // U_re from S_re
      IY1[size_t(y) * 4 * m + 2 * kyi + 1] = -s;  // U_re from S_im
      IY2[size_t(y) * 4 * m + 2 * kyi] = s;       // U_im from S_re
      IY2[size_t(y) * 4 * m + 2 * kyi + 1] = c;   // U_im from S_im
    }
  }
  std::vector<double> FxT(size_t(2 * m) * W);  // Fx transposed: [2kx+p][x]
  for (int x = 0; x < W; ++x)
    for (int j = 0; j < 2 * m; ++j) FxT[size_t(j) * W + x] = Fx[size_t(x) * 2 * m + j];
  qla_status st = upload16(f, &f->Fx, Fx);
  if (st == QLA_OK) st = upload16(f, &f->FxT, FxT);
  if (st == QLA_OK) st = upload16(f, &f->IX, IX);
  if (st == QLA_OK) st = upload16(f, &f->A1, A1);
  if (st == QLA_OK) st = upload16(f, &f->A2, A2);
  std::vector<double> IY1T(IY1.size()), IY2T(IY2.size());  // [2kyi + p'][y]
  for (int y = 0; y < H; ++y)
    for (int k = 0; k < 4 * m; ++k) {
      IY1T[size_t(k) * H + y] = IY1[size_t(y) * 4 * m + k];
      IY2T[size_t(k) * H + y] = IY2[size_t(y) * 4 * m + k];
    }
  if (st == QLA_OK) st = upload16(f, &f->IY1T, IY1T);
  if (st == QLA_OK) st = upload16(f, &f->IY2T, IY2T);
  std::vector<double> A1T(A1.size()), A2T(A2.size());  // [y][2kyi + p']
  for (int k = 0; k < 4 * m; ++k)
    for (int y = 0; y < H; ++y) {
      A1T[size_t(y) * 4 * m + k] = A1[size_t(k) * H + y];
      A2T[size_t(y) * 4 * m + k] = A2[size_t(k) * H + y];
    }
  if (st == QLA_OK) st = upload16(f, &f->A1T, A1T);
  if (st == QLA_OK) st = upload16(f, &f->A2T, A2T);
  if (st == QLA_OK) st = upload16(f, &f->IY1, IY1);
  if (st == QLA_OK) st = upload16(f, &f->IY2, IY2);
  return st;
}

// BF16 copies of the GEMM weights from the FP32 master parameters.
qla_status refresh_w16(qla_fno* f) {
  auto cast = [&](size_t off, size_t dst, size_t n) -> hipError_t {
    hipLaunchKernelGGL(cast_kernel, dim3(grid_for(n)), dim3(kBlock), 0, f->stream, f->p + off,
                       f->w16 + dst, n);
    return hipGetLastError();
  };
  QLA_HIP(cast(f->o_Wp, f->w16_Wp(), size_t(f->C) * f->Cin));
  for (int l = 0; l < f->L; ++l) QLA_HIP(cast(f->o_W[l], f->w16_W(l), size_t(f->C) * f->C));
  QLA_HIP(cast(f->o_Q1, f->w16_Q1(), size_t(f->C2) * f->C));
  QLA_HIP(cast(f->o_Q2, f->w16_Q2(), size_t(f->Cout) * f->C2));
  return QLA_OK;
}

// Per-sample 1x1 convolution: out[b][mo][p] = sum_k Wt[mo][k] in[b][k][p] (weights
// row-major mo x k, or transposed when wt_t).
GemmDesc pointwise(const uint16_t* wt, bool wt_t, int Mo, int K, const uint16_t* in, int B,
                   size_t P) {
  GemmDesc g;
  g.A = wt;
  g.sAb = 0;
  g.sAm = wt_t ? 1 : K;
  g.sAk = wt_t ? Mo : 1;
  g.B = in;
  g.sBb = static_cast<long long>(K) * P;
  g.sBk = static_cast<long long>(P);
  g.sBn = 1;
  g.sCb = static_cast<long long>(Mo) * P;
  g.sCm = static_cast<long long>(P);
  g.sCn = 1;
  g.M = Mo;
  g.N = static_cast<int>(P);
  g.K = K;
  g.batch = B;
  return g;
}

// Weight gradient dWt[mo][k] += sum_{b,p} d[b][mo][p] x[b][k][p] (split over pixels);
// the bias gradient db[mo] += sum_{b,p} d[b][mo][p] comes out of the same launch.
GemmDesc weight_grad(const uint16_t* d, int Mo, const uint16_t* x, int K, int B, size_t P,
                     float* dW, float* db) {
  GemmDesc g;
  g.A = d;
  g.sAb = static_cast<long long>(Mo) * P;
  g.sAm = static_cast<long long>(P);
  g.sAk = 1;
  g.B = x;
  g.sBb = static_cast<long long>(K) * P;
  g.sBk = 1;
  g.sBn = static_cast<long long>(P);
  g.C = dW;
  g.sCb = 0;
  g.sCm = K;
  g.sCn = 1;
  g.M = Mo;
  g.N = K;
  g.K = static_cast<int>(P);
  g.batch = B;
  // 1024-pixel splits (at most 256 per sample): measured against 2048-, 4096- and 8192-pixel
  // splits at 512^2, batch 16 (training 1754 samples/s against 1731, 1657 and 1750)
  g.ksplit = static_cast<int>(std::max<size_t>(1, std::min<size_t>(256, P / 1024)));
  g.atomic = 1;
  g.rowsum = db;
  return g;
}

#define QLA_GEMM(desc) QLA_HIP(qla::fno::launch_gemm((desc), f->stream))

// dW (Mo x K) += d x^T and db += d 1 over the batch: the matrix-core weight-gradient kernel
// where the channel counts fit it, else the split GEMM.
hipError_t weight_grad_run(const qla_fno* f, const uint16_t* d, int Mo, const uint16_t* x, int K,
                           int B, float* dW, float* db) {
  int mh = 0, nh = 0;
  if (wgrad_shape(Mo, K, f->P, &mh, &nh))
    return launch_wgrad(d, Mo, x, K, B, f->P, f->cus, f->wpart, dW, db, f->stream);
  return qla::fno::launch_gemm(weight_grad(d, Mo, x, K, B, f->P, dW, db), f->stream);
}

// The inverse x transform of the spectral branch as a second contraction of the
// channel-mixing GEMM g (whose columns are pixels): adds sum_j U[(b,o), y][j] IX[j][x].
void add_inverse_x(const qla_fno* f, GemmDesc* g) {
  g->A2 = f->Ub;
  g->sA2b = static_cast<long long>(f->C) * f->H * 2 * f->m;
  g->sA2m = static_cast<long long>(f->H) * 2 * f->m;
  g->sA2y = 2 * f->m;
  g->sA2k = 1;
  g->B2 = f->IX;
  g->sB2k = f->W;
  g->sB2x = 1;
  g->K2 = 2 * f->m;
  g->row = f->W;
}

// The backward counterpart: adds sum_j dZ[(b,c), y][j] Fx[x][j].
void add_forward_x_transposed(const qla_fno* f, GemmDesc* g) {
  g->A2 = f->dZ;
  g->sA2b = static_cast<long long>(f->C) * f->H * 2 * f->m;
  g->sA2m = static_cast<long long>(f->H) * 2 * f->m;
  g->sA2y = 2 * f->m;
  g->sA2k = 1;
  g->B2 = f->Fx;
  g->sB2k = 1;
  g->sB2x = 2 * f->m;
  g->K2 = 2 * f->m;
  g->row = f->W;
}

// Forward pass of batch B: input BF16 [B][Cin][P] -> f->out FP32 [B][Cout][P].
// `training` keeps the pre-activations the backward pass needs.
qla_status forward(qla_fno* f, const uint16_t* in, int B, bool training) {
  const size_t P = f->P;
  const int C = f->C, H = f->H, W = f->W, m = f->m;
  const long long modes_sz = 4LL * m * m;  // floats per (b, c) in T, S
  // lift
  if (f->Cin <= kLiftMaxIn && C <= kLiftMaxC) {
    const long long threads = (static_cast<long long>(P) + 7) / 8 * B;
    const long long blocks = (threads + 255) / 256;
    hipLaunchKernelGGL(lift_kernel, dim3(static_cast<unsigned>(blocks < 8192 ? blocks : 8192)),
                       dim3(256), 0, f->stream, in, f->w16 + f->w16_Wp(), f->p + f->o_bp, f->Cin,
                       C, static_cast<long long>(P), B, f->v[0]);
    QLA_HIP(hipGetLastError());
  } else {
    GemmDesc g = pointwise(f->w16 + f->w16_Wp(), false, C, f->Cin, in, B, P);
    g.C = f->v[0];
    g.out_bf16 = 1;
    g.bias = f->p + f->o_bp;
    QLA_GEMM(g);
  }
  for (int l = 0; l < f->L; ++l) {
    const uint16_t* vl = f->v[l];
    if (spectral_in_fits(H, W, m)) {
      // x and y transforms in one pass: T[l] straight from v
      QLA_HIP(launch_spectral_in(vl, static_cast<long long>(C) * P, static_cast<long long>(P), C,
                                 B * C, f->FxT, f->A1, f->A2, H, W, m, f->T[l], f->stream));
    } else {
      // x transform: Z[(b,c,y)][2kx+p]
      {
        GemmDesc g;
        g.A = vl;
        g.sAm = W;
        g.sAk = 1;
        g.B = f->Fx;
        g.sBk = 2 * m;
        g.sBn = 1;
        g.C = f->Zb;
        g.sCm = 2 * m;
        g.sCn = 1;
        g.M = B * C * H;
        g.N = 2 * m;
        g.K = W;
        g.out_bf16 = 1;
        QLA_GEMM(g);
      }
      // y transform: T[(b,c)] = A1 Zre + A2 Zim
      for (int part = 0; part < 2; ++part) {
        GemmDesc g;
        g.A = part ? f->A2 : f->A1;
        g.sAm = H;
        g.sAk = 1;
        g.B = f->Zb + part;
        g.sBb = static_cast<long long>(H) * 2 * m;
        g.sBk = 2 * m;
        g.sBn = 2;
        g.C = f->T[l];
        g.sCb = modes_sz;
        g.sCm = m;
        g.sCn = 1;
        g.M = 4 * m;
        g.N = m;
        g.K = H;
        g.batch = B * C;
        g.beta = part;
        QLA_GEMM(g);
      }
    }
    hipLaunchKernelGGL(mix_forward_kernel, dim3(2 * m * m, kModeSplit), dim3(256), 0, f->stream, f->T[l],
                       f->p + f->o_R[l], f->Sb, B, C, m);
    QLA_HIP(hipGetLastError());
    // inverse y: U[(b,o)][y][2kx+p] = IY_p S
    if (spectral_out_fits(m)) {
      QLA_HIP(launch_spectral_out(f->Sb, f->IY1, f->IY2, B * C, H, m, f->Ub, f->stream));
    } else {
      for (int part = 0; part < 2; ++part) {
        GemmDesc g;
        g.A = part ? f->IY2 : f->IY1;
        g.sAm = 4 * m;
        g.sAk = 1;
        g.B = f->Sb;
        g.sBb = modes_sz;
        g.sBk = m;
        g.sBn = 1;
        g.C = f->Ub + part;
        g.sCb = static_cast<long long>(H) * 2 * m;
        g.sCm = 2 * m;
        g.sCn = 2;
        g.M = H;
        g.N = m;
        g.K = 4 * m;
        g.batch = B * C;
        g.out_bf16 = 1;
        QLA_GEMM(g);
      }
    }
    if (!f->fused) {
      // inverse x: spec[(b,o,y)][x]
      GemmDesc g;
      g.A = f->Ub;
      g.sAm = 2 * m;
      g.sAk = 1;
      g.B = f->IX;
      g.sBk = W;
      g.sBn = 1;
      g.C = f->spec;
      g.sCm = W;
      g.sCn = 1;
      g.M = B * C * H;
      g.N = W;
      g.K = 2 * m;
      QLA_GEMM(g);
    }
    // pointwise + spectral + bias, then GELU (not after the last layer)
    if (f->fused && C == kMixC && W % kMixPix == 0 && 2 * m <= kMixMaxJ) {
      // a multiple of the tiles per grid row, so every block keeps one column range (and
      // its slice of the inverse x basis) for all its tiles
      const long long per_row = W / kMixPix;
      const long long tiles = static_cast<long long>(B) * H * per_row;
      const long long nb = tiles < 1024 ? tiles : 1024;
      const dim3 grid(static_cast<unsigned>(nb >= per_row ? nb / per_row * per_row : per_row));
      const bool last = l + 1 == f->L;
      uint16_t* zo = last ? f->v[l + 1] : (training ? f->z[l] : nullptr);
      uint16_t* ao = last ? nullptr : f->v[l + 1];
      hipLaunchKernelGGL(layer_mix_kernel<false>, grid, dim3(256), 0, f->stream, vl,
                         f->w16 + f->w16_W(l), f->p + f->o_b[l], f->Ub, f->IX, 2 * m, H, W, B,
                         zo, ao, nullptr);
      QLA_HIP(hipGetLastError());
    } else {
      GemmDesc g = pointwise(f->w16 + f->w16_W(l), false, C, C, vl, B, P);
      g.bias = f->p + f->o_b[l];
      if (f->fused) {
        add_inverse_x(f, &g);
      } else {
        g.res = f->spec;
        g.sRb = static_cast<long long>(C) * P;
        g.sRm = static_cast<long long>(P);
        g.sRn = 1;
      }
      g.out_bf16 = 1;
      if (l + 1 < f->L) {
        g.C = training ? f->z[l] : nullptr;
        g.act = f->v[l + 1];
      } else {
        g.C = f->v[l + 1];
      }
      QLA_GEMM(g);
    }
  }
  // projection: h = GELU(Q1 v_L + bq1), out = Q2 h + bq2 (inference: in one pass)
  if (!training && C <= kProjMaxC && f->C2 <= kProjMaxC2 && f->Cout <= kProjMaxOut) {
    // enough blocks to fill the chip several times over; each strides over tiles
    const long long tiles = (static_cast<long long>(P) + kProjPix - 1) / kProjPix * B;
    const dim3 grid(static_cast<unsigned>(tiles < 4096 ? tiles : 4096));
    hipLaunchKernelGGL(projection_fused_kernel, grid, dim3(256), 0, f->stream, f->v[f->L], f->w16 + f->w16_Q1(), f->p + f->o_bq1,
                       f->w16 + f->w16_Q2(), f->p + f->o_bq2, C, f->C2, f->Cout,
                       static_cast<long long>(P), B, f->out);
    QLA_HIP(hipGetLastError());
    return QLA_OK;
  }
  if (training && C == kMixC && W % kMixPix == 0 && f->C2 % kMixC == 0 &&
      f->C2 <= kProj1MaxGroups * kMixC) {
    // one resident round of blocks (two per compute unit), each striding over tiles
    const long long tiles = static_cast<long long>(B) * H * (W / kMixPix);
    const long long want = 2LL * std::max(f->cus, 1);
    // the second projection in the same pass where it is narrow (h is then not read back)
    const bool with_out = f->Cout <= kNarrowOut;
    hipLaunchKernelGGL(proj1_train_kernel, dim3(static_cast<unsigned>(std::min(tiles, want))),
                       dim3(256), 0, f->stream, f->v[f->L], f->w16 + f->w16_Q1(),
                       f->p + f->o_bq1, f->C2 / kMixC, H, W, B, f->zq, f->h,
                       f->w16 + f->w16_Q2(), f->p + f->o_bq2, f->Cout,
                       with_out ? f->out : nullptr);
    QLA_HIP(hipGetLastError());
    if (with_out) return QLA_OK;
  } else {
    GemmDesc g = pointwise(f->w16 + f->w16_Q1(), false, f->C2, C, f->v[f->L], B, P);
    g.bias = f->p + f->o_bq1;
    g.C = training ? f->zq : nullptr;
    g.out_bf16 = 1;
    g.act = f->h;
    QLA_GEMM(g);
  }
  if (f->Cout <= kNarrowOut && f->C2 <= kNarrowC2 && P % 8 == 0) {
    const long long threads = static_cast<long long>(P) / 8 * B;
    const long long blocks = (threads + 255) / 256;
    hipLaunchKernelGGL(narrow_projection_kernel,
                       dim3(static_cast<unsigned>(blocks < 8192 ? blocks : 8192)), dim3(256), 0,
                       f->stream, f->h, f->w16 + f->w16_Q2(), f->p + f->o_bq2, f->C2, f->Cout,
                       static_cast<long long>(P), B, f->out);
    QLA_HIP(hipGetLastError());
  } else {
    GemmDesc g = pointwise(f->w16 + f->w16_Q2(), false, f->Cout, f->C2, f->h, B, P);
    g.bias = f->p + f->o_bq2;
    g.C = f->out;
    QLA_GEMM(g);
  }
  return QLA_OK;
}

// Loss and gradients of the batch (forward(training) must have run on `in`).
// Gradients are accumulated into f->g, which the caller zeroes.
qla_status backward(qla_fno* f, const uint16_t* in, const uint16_t* target, int B) {
  const size_t P = f->P;
  const int C = f->C, C2 = f->C2, H = f->H, W = f->W, m = f->m, L = f->L;
  const size_t per = size_t(f->Cout) * P;
  const long long modes_sz = 4LL * m * m;
  hipLaunchKernelGGL(loss_partial_kernel, dim3(kLossBlocks, B), dim3(kBlock), 0, f->stream,
                     f->out, target, f->lpart, per);
  QLA_HIP(hipGetLastError());
  hipLaunchKernelGGL(loss_sums_kernel, dim3((2 * B + 63) / 64), dim3(64), 0, f->stream, f->lpart,
                     kLossBlocks, B, f->sums);
  QLA_HIP(hipGetLastError());
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, f->stream, f->sums, B, f->loss);
  QLA_HIP(hipGetLastError());
  hipLaunchKernelGGL(loss_grad_kernel, dim3(256, B), dim3(kBlock), 0, f->stream, f->out, target,
                     f->sums, f->dout, B, per);
  QLA_HIP(hipGetLastError());
  // projection 2, then dzq = (Q2^T dout) GELU'(zq)
  QLA_HIP(weight_grad_run(f, f->dout, f->Cout, f->h, C2, B, f->g + f->o_Q2, f->g + f->o_bq2));
  uint16_t* dz = f->dza;       // gradient with respect to z_l
  uint16_t* dz_prev = f->dzb;  // gradient with respect to z_{l-1} (or v_0)
  if (C == kMixC && W % kMixPix == 0 && C2 % kMixC == 0 && C2 <= kProj1MaxGroups * kMixC &&
      f->Cout <= kNarrowOut) {
    // dzq and dz_{L-1} = Q1^T dzq in one pass (no activation after the last layer)
    const long long tiles = static_cast<long long>(B) * H * (W / kMixPix);
    const long long want = 2LL * std::max(f->cus, 1);
    hipLaunchKernelGGL(proj_grad_kernel, dim3(static_cast<unsigned>(std::min(tiles, want))),
                       dim3(256), 0, f->stream, f->dout, f->w16 + f->w16_Q2(), f->zq,
                       f->w16 + f->w16_Q1(), C2 / kMixC, f->Cout, H, W, B, f->dzq, dz);
    QLA_HIP(hipGetLastError());
    QLA_HIP(weight_grad_run(f, f->dzq, C2, f->v[L], C, B, f->g + f->o_Q1, f->g + f->o_bq1));
  } else {
    if (f->Cout <= kNarrowOut && C2 <= kNarrowC2 && P % 8 == 0) {
      const long long threads = static_cast<long long>(P) / 8 * B;
      const long long blocks = (threads + 255) / 256;
      hipLaunchKernelGGL(narrow_projection_grad_kernel,
                         dim3(static_cast<unsigned>(blocks < 8192 ? blocks : 8192)), dim3(256),
                         0, f->stream, f->dout, f->w16 + f->w16_Q2(), f->zq, C2, f->Cout,
                         static_cast<long long>(P), B, f->dzq);
      QLA_HIP(hipGetLastError());
    } else {
      GemmDesc g = pointwise(f->w16 + f->w16_Q2(), true, C2, f->Cout, f->dout, B, P);
      g.C = f->dzq;
      g.out_bf16 = 1;
      g.gz = f->zq;
      QLA_GEMM(g);
    }
    // projection 1, then dz_{L-1} = Q1^T dzq (no activation after the last layer)
    QLA_HIP(weight_grad_run(f, f->dzq, C2, f->v[L], C, B, f->g + f->o_Q1, f->g + f->o_bq1));
    GemmDesc g = pointwise(f->w16 + f->w16_Q1(), true, C, C2, f->dzq, B, P);
    g.C = dz;
    g.out_bf16 = 1;
    QLA_GEMM(g);
  }
  for (int l = L - 1; l >= 0; --l) {
    const uint16_t* vl = f->v[l];
    QLA_HIP(weight_grad_run(f, dz, C, vl, C, B, f->g + f->o_W[l], f->g + f->o_b[l]));
    // spectral branch: dS = IY1^T dUre + IY2^T dUim with dU = dz IX^T, in one pass over dz
    // (the forward's x and y transform kernel with IX for the x basis and the transposed
    // inverse y bases), or as the two products below
    if (spectral_in_fits(H, W, m)) {
      QLA_HIP(launch_spectral_in(dz, static_cast<long long>(C) * P, static_cast<long long>(P), C,
                                 B * C, f->IX, f->IY1T, f->IY2T, H, W, m, f->dS, f->stream,
                                 true));
    } else {
      {
        GemmDesc g;
        g.A = dz;
        g.sAm = W;
        g.sAk = 1;
        g.B = f->IX;
        g.sBk = 1;
        g.sBn = W;
        g.C = f->dU;
        g.sCm = 2 * m;
        g.sCn = 1;
        g.M = B * C * H;
        g.N = 2 * m;
        g.K = W;
        g.out_bf16 = 1;
        QLA_GEMM(g);
      }
      // dS = IY1^T dUre + IY2^T dUim
      if (spectral_out_fits(m)) {
        QLA_HIP(launch_spectral_y(f->dU, f->IY1T, f->IY2T, B * C, H, m, f->dS, f->stream));
      } else {
        for (int part = 0; part < 2; ++part) {
          GemmDesc g;
          g.A = part ? f->IY2 : f->IY1;
          g.sAm = 1;
          g.sAk = 4 * m;
          g.B = f->dU + part;
          g.sBb = static_cast<long long>(H) * 2 * m;
          g.sBk = 2 * m;
          g.sBn = 2;
          g.C = f->dS;  // mode-major: [2kyi + p][kx][(b, o)]
          g.sCb = 1;
          g.sCm = static_cast<long long>(m) * B * C;
          g.sCn = static_cast<long long>(B) * C;
          g.M = 4 * m;
          g.N = m;
          g.K = H;
          g.batch = B * C;
          g.beta = part;
          QLA_GEMM(g);
        }
      }
    }
    hipLaunchKernelGGL(mix_backward_weight_kernel, dim3(2 * m * m, kModeSplit), dim3(256), 0, f->stream,
                       f->dS, f->T[l], f->g + f->o_R[l], B, C, m);
    QLA_HIP(hipGetLastError());
    hipLaunchKernelGGL(mix_backward_input_kernel, dim3(2 * m * m, kModeSplit), dim3(256), 0, f->stream,
                       f->dS, f->p + f->o_R[l], f->dT, B, C, m);
    QLA_HIP(hipGetLastError());
    // dZ_p = A_p^T dT  (p = re, im)
    if (spectral_out_fits(m)) {
      QLA_HIP(launch_spectral_out(f->dT, f->A1T, f->A2T, B * C, H, m, f->dZ, f->stream));
    } else {
      for (int part = 0; part < 2; ++part) {
        GemmDesc g;
        g.A = part ? f->A2 : f->A1;
        g.sAm = 1;
        g.sAk = H;
        g.B = f->dT;
        g.sBb = modes_sz;
        g.sBk = m;
        g.sBn = 1;
        g.C = f->dZ + part;
        g.sCb = static_cast<long long>(H) * 2 * m;
        g.sCm = 2 * m;
        g.sCn = 2;
        g.M = H;
        g.N = m;
        g.K = 4 * m;
        g.batch = B * C;
        g.out_bf16 = 1;
        QLA_GEMM(g);
      }
    }
    // dv_l = W_l^T dz + dZ Fx^T; dz_{l-1} = dv_l GELU'(z_{l-1}) (v_0 has no activation)
    const uint16_t* gz = l > 0 ? f->z[l - 1] : nullptr;
    if (f->fused && C == kMixC && W % kMixPix == 0 && 2 * m <= kMixMaxJ) {
      // the layer kernel's backward mode (same grid as forward)
      const long long per_row = W / kMixPix;
      const long long tiles = static_cast<long long>(B) * H * per_row;
      const long long nb = tiles < 1024 ? tiles : 1024;
      const dim3 grid(static_cast<unsigned>(nb >= per_row ? nb / per_row * per_row : per_row));
      hipLaunchKernelGGL(layer_mix_kernel<true>, grid, dim3(256), 0, f->stream, dz,
                         f->w16 + f->w16_W(l), nullptr, f->dZ, f->Fx, 2 * m, H, W, B, dz_prev,
                         nullptr, gz);
      QLA_HIP(hipGetLastError());
      std::swap(dz, dz_prev);
      continue;
    }
    GemmDesc g = pointwise(f->w16 + f->w16_W(l), true, C, C, dz, B, P);
    if (f->fused) {
      add_forward_x_transposed(f, &g);
      g.C = dz_prev;
      g.out_bf16 = 1;
      g.gz = gz;
      QLA_GEMM(g);
    } else {
      g.C = f->dv;
      QLA_GEMM(g);
      GemmDesc h;
      h.A = f->dZ;
      h.sAm = 2 * m;
      h.sAk = 1;
      h.B = f->Fx;
      h.sBk = 1;
      h.sBn = 2 * m;
      h.C = f->dv;
      h.sCm = W;
      h.sCn = 1;
      h.M = B * C * H;
      h.N = W;
      h.K = 2 * m;
      h.beta = 1;
      QLA_GEMM(h);
      const size_t nact = size_t(B) * C * P;
      if (gz) {
        hipLaunchKernelGGL(gelu_grad_kernel, dim3(grid_for(nact)), dim3(kBlock), 0, f->stream,
                           f->dv, gz, dz_prev, nact);
      } else {
        hipLaunchKernelGGL(cast_kernel, dim3(grid_for(nact)), dim3(kBlock), 0, f->stream, f->dv,
                           dz_prev, nact);
      }
      QLA_HIP(hipGetLastError());
    }
    std::swap(dz, dz_prev);
  }
  // lift (dz now holds the gradient with respect to v_0)
  QLA_HIP(weight_grad_run(f, dz, C, in, f->Cin, B, f->g + f->o_Wp, f->g + f->o_bp));
  return QLA_OK;
}

qla_status check_batch(const qla_fno* f, int B) {
  if (B < 1 || B > f->Bmax) return fail(QLA_EINVAL, "batch must be in [1, max_batch]");
  return QLA_OK;
}

}  // namespace

extern "C" {

qla_status qla_fno_create(int height, int width, int in_channels, int out_channels, int channels,
                          int modes, int layers, int proj_channels, int max_batch, uint64_t seed,
                          void* hip_stream, qla_fno** out) {
  if (!out) return fail(QLA_EINVAL, "out is NULL");
  *out = nullptr;
  if (height < 2 || width < 2 || in_channels < 1 || out_channels < 1 || channels < 1 ||
      modes < 1 || layers < 1 || proj_channels < 1 || max_batch < 1)
    return fail(QLA_EINVAL, "sizes must be positive");
  if (2 * modes > height || 2 * modes > width)
    return fail(QLA_EINVAL, "need 2 * modes <= height and 2 * modes <= width");
  if (channels > kModeC)
    return fail(QLA_EINVAL, "channels must be <= " + std::to_string(kModeC));
  if (static_cast<long long>(max_batch) * std::max(channels, proj_channels) * height * width >=
      (1ll << 31))
    return fail(QLA_EINVAL, "max_batch * channels * height * width must be < 2^31");
  qla_fno* f = new (std::nothrow) qla_fno;
  if (!f) return fail(QLA_ENOMEM, "host allocation");
  f->H = height;
  f->W = width;
  f->P = height * width;
  f->Cin = in_channels;
  f->Cout = out_channels;
  f->C = channels;
  f->C2 = proj_channels;
  f->L = layers;
  f->m = modes;
  f->Bmax = max_batch;
  hipError_t e = hipGetDevice(&f->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&f->cus, hipDeviceAttributeMultiprocessorCount, f->device);
  if (e == hipSuccess && hip_stream) {
    f->stream = static_cast<hipStream_t>(hip_stream);
  } else if (e == hipSuccess) {
    e = hipStreamCreateWithFlags(&f->stream, hipStreamNonBlocking);
    f->own_stream = e == hipSuccess;
  }
  if (e != hipSuccess) {
    delete f;
    return hip_fail(e, "stream");
  }
  // parameter layout
  const int C = channels, m = modes;
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t o = off;
    off += n;
    return o;
  };
  f->o_Wp = take(size_t(C) * in_channels);
  f->o_bp = take(C);
  for (int l = 0; l < layers; ++l) {
    f->o_W.push_back(take(size_t(C) * C));
    f->o_b.push_back(take(C));
    f->o_R.push_back(take(size_t(2 * m * m) * C * C * 2));
  }
  f->o_Q1 = take(size_t(proj_channels) * C);
  f->o_bq1 = take(proj_channels);
  f->o_Q2 = take(size_t(out_channels) * proj_channels);
  f->o_bq2 = take(out_channels);
  f->nparam = off;
  f->nweights16 = size_t(C) * in_channels + size_t(layers) * C * C + size_t(proj_channels) * C +
                  size_t(out_channels) * proj_channels;
  const size_t B = max_batch, P = f->P;
  qla_status st = QLA_OK;
  auto A = [&](auto** p, size_t n) {
    if (st == QLA_OK) st = dalloc_t(f, p, n);
  };
  A(&f->p, f->nparam);
  A(&f->g, f->nparam);
  A(&f->m1, f->nparam);
  A(&f->m2, f->nparam);
  A(&f->w16, f->nweights16);
  f->v.assign(layers + 1, nullptr);
  f->z.assign(layers, nullptr);
  f->T.assign(layers, nullptr);
  for (int l = 0; l <= layers; ++l) A(&f->v[l], B * C * P);
  for (int l = 0; l + 1 < layers; ++l) A(&f->z[l], B * C * P);
  for (int l = 0; l < layers; ++l) A(&f->T[l], B * C * 4 * m * m);
  A(&f->Zb, B * C * height * 2 * m);
  A(&f->Sb, B * C * 4 * m * m);
  A(&f->Ub, B * C * height * 2 * m);
  f->fused = width % 64 == 0;
  if (!f->fused) {
    A(&f->spec, B * C * P);
    A(&f->dv, B * C * P);
  }
  A(&f->zq, B * proj_channels * P);
  A(&f->h, B * proj_channels * P);
  A(&f->out, B * out_channels * P);
  A(&f->dout, B * out_channels * P);
  A(&f->dzq, B * proj_channels * P);
  A(&f->dza, B * C * P);
  A(&f->dzb, B * C * P);
  A(&f->dU, B * C * height * 2 * m);
  A(&f->dS, B * C * 4 * m * m);
  A(&f->dT, B * C * 4 * m * m);
  A(&f->dZ, B * C * height * 2 * m);
  A(&f->wpart, size_t(kWgBlocks) * kWgMaxE);
  A(&f->loss, 1);
  A(&f->sums, 2 * B);
  A(&f->lpart, 2 * B * kLossBlocks);
  A(&f->band, 2 * B);
  if (st == QLA_OK) st = make_bases(f);
  if (st != QLA_OK) {
    release(f);
    delete f;
    return st;
  }
  // initial weights: linear maps U(-1/sqrt(fan_in), 1/sqrt(fan_in)); spectral weights
  // 1/(C*C) times U(0, 1) for both parts
  std::vector<float> hp(f->nparam);
  Rng rng{seed};
  auto lin = [&](size_t o, size_t n, int fan_in) {
    const double a = 1.0 / std::sqrt(double(fan_in));
    for (size_t i = 0; i < n; ++i) hp[o + i] = static_cast<float>((2.0 * rng.uniform() - 1.0) * a);
  };
  lin(f->o_Wp, size_t(C) * in_channels, in_channels);
  lin(f->o_bp, C, in_channels);
  for (int l = 0; l < layers; ++l) {
    lin(f->o_W[l], size_t(C) * C, C);
    lin(f->o_b[l], C, C);
    const size_t n = size_t(2 * m * m) * C * C * 2;
    for (size_t i = 0; i < n; ++i) hp[f->o_R[l] + i] = static_cast<float>(rng.uniform() / (double(C) * C));
  }
  lin(f->o_Q1, size_t(proj_channels) * C, C);
  lin(f->o_bq1, proj_channels, C);
  lin(f->o_Q2, size_t(out_channels) * proj_channels, proj_channels);
  lin(f->o_bq2, out_channels, proj_channels);
  e = hipMemcpy(f->p, hp.data(), hp.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(f->m1, 0, f->nparam * sizeof(float));
  if (e == hipSuccess) e = hipMemset(f->m2, 0, f->nparam * sizeof(float));
  if (e == hipSuccess) e = hipMemset(f->g, 0, f->nparam * sizeof(float));
  if (e != hipSuccess) {
    release(f);
    delete f;
    return hip_fail(e, "FNO initialisation");
  }
  st = refresh_w16(f);
  if (st == QLA_OK) {
    e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
  }
  if (st != QLA_OK) {
    release(f);
    delete f;
    return st;
  }
  *out = f;
  return QLA_OK;
}

qla_status qla_fno_destroy(qla_fno* f) {
  if (!f) return QLA_OK;
  DeviceGuard g(f->device);  // frees what it can even if selecting the device fails
  if (f->stream) (void)hipStreamSynchronize(f->stream);
  release(f);
  delete f;
  return QLA_OK;
}

qla_status qla_fno_param_count(const qla_fno* f, int64_t* count) {
  if (!f || !count) return fail(QLA_EINVAL, "NULL argument");
  *count = static_cast<int64_t>(f->nparam);
  return QLA_OK;
}

qla_status qla_fno_get_params(qla_fno* f, float* host) {
  if (!f || !host) return fail(QLA_EINVAL, "NULL argument");
  QLA_ON_DEVICE(f->device);
  QLA_HIP(hipMemcpyAsync(host, f->p, f->nparam * sizeof(float), hipMemcpyDeviceToHost, f->stream));
  QLA_HIP(hipStreamSynchronize(f->stream));
  return QLA_OK;
}

qla_status qla_fno_set_params(qla_fno* f, const float* host) {
  if (!f || !host) return fail(QLA_EINVAL, "NULL argument");
  QLA_ON_DEVICE(f->device);
  QLA_HIP(hipMemcpyAsync(f->p, host, f->nparam * sizeof(float), hipMemcpyHostToDevice, f->stream));
  qla_status st = refresh_w16(f);
  if (st != QLA_OK) return st;
  QLA_HIP(hipStreamSynchronize(f->stream));
  return QLA_OK;
}

qla_status qla_fno_get_grads(qla_fno* f, float* host) {
  if (!f || !host) return fail(QLA_EINVAL, "NULL argument");
  QLA_ON_DEVICE(f->device);
  QLA_HIP(hipMemcpyAsync(host, f->g, f->nparam * sizeof(float), hipMemcpyDeviceToHost, f->stream));
  QLA_HIP(hipStreamSynchronize(f->stream));
  return QLA_OK;
}

qla_status qla_fno_forward(qla_fno* f, const uint16_t* input, int batch, float* output) {
  if (!f || !input || !output) return fail(QLA_EINVAL, "NULL argument");
  qla_status st = check_batch(f, batch);
  if (st != QLA_OK) return st;
  QLA_ON_DEVICE(f->device);
  st = forward(f, input, batch, false);
  if (st != QLA_OK) return st;
  QLA_HIP(hipMemcpyAsync(output, f->out, size_t(batch) * f->Cout * f->P * sizeof(float),
                         hipMemcpyDeviceToDevice, f->stream));
  return QLA_OK;
}

qla_status qla_fno_loss_grad(qla_fno* f, const uint16_t* input, const uint16_t* target, int batch,
                             float* loss_host) {
  if (!f || !input || !target) return fail(QLA_EINVAL, "NULL argument");
  qla_status st = check_batch(f, batch);
  if (st != QLA_OK) return st;
  QLA_ON_DEVICE(f->device);
  QLA_HIP(hipMemsetAsync(f->g, 0, f->nparam * sizeof(float), f->stream));
  st = forward(f, input, batch, true);
  if (st == QLA_OK) st = backward(f, input, target, batch);
  if (st != QLA_OK) return st;
  if (loss_host) {
    QLA_HIP(hipMemcpyAsync(loss_host, f->loss, sizeof(float), hipMemcpyDeviceToHost, f->stream));
    QLA_HIP(hipStreamSynchronize(f->stream));
  }
  return QLA_OK;
}

qla_status qla_fno_adam_step(qla_fno* f, float lr, float beta1, float beta2, float eps) {
  if (!f) return fail(QLA_EINVAL, "NULL argument");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(QLA_EINVAL, "bad Adam hyper-parameters");
  QLA_ON_DEVICE(f->device);
  ++f->adam_t;
  const float c1 = static_cast<float>(1.0 / (1.0 - std::pow(double(beta1), double(f->adam_t))));
  const float c2 = static_cast<float>(1.0 / (1.0 - std::pow(double(beta2), double(f->adam_t))));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(f->nparam)), dim3(kBlock), 0, f->stream, f->p, f->g,
                     f->m1, f->m2, f->nparam, lr, beta1, beta2, eps, c1, c2);
  QLA_HIP(hipGetLastError());
  return refresh_w16(f);
}

qla_status qla_fno_train_step(qla_fno* f, const uint16_t* input, const uint16_t* target,
                              int batch, float lr, float* loss_device) {
  qla_status st = qla_fno_loss_grad(f, input, target, batch, nullptr);
  if (st != QLA_OK) return st;
  if (loss_device) {
    QLA_ON_DEVICE(f->device);
    QLA_HIP(hipMemcpyAsync(loss_device, f->loss, sizeof(float), hipMemcpyDeviceToDevice,
                           f->stream));
  }
  return qla_fno_adam_step(f, lr, 0.9f, 0.999f, 1e-8f);
}

qla_status qla_fno_band_fraction(qla_fno* f, const uint16_t* input, int batch, int first_channel,
                                 int channels, double* fraction_device) {
  if (!f || !input || !fraction_device) return fail(QLA_EINVAL, "NULL argument");
  qla_status st = check_batch(f, batch);
  if (st != QLA_OK) return st;
  if (first_channel < 0 || channels < 1 || channels > f->C ||
      first_channel + channels > f->Cin)
    return fail(QLA_EINVAL, "channels must lie within the input planes (at most C of them)");
  QLA_ON_DEVICE(f->device);
  const int H = f->H, W = f->W, m = f->m;
  const size_t P = f->P;
  // the truncated transforms of a Fourier layer, applied to the chosen input planes,
  // into the forward pass's transform scratch (every forward pass rewrites it)
  const uint16_t* planes = input + size_t(first_channel) * P;
  if (spectral_in_fits(H, W, m) && (reinterpret_cast<uintptr_t>(planes) & 15) == 0) {
    QLA_HIP(launch_spectral_in(planes, static_cast<long long>(f->Cin) * P,
                               static_cast<long long>(P), channels, batch * channels, f->FxT,
                               f->A1, f->A2, H, W, m, f->T[0], f->stream));
  } else {
    {
      GemmDesc g;
      g.A = input + size_t(first_channel) * P;
      g.sAb = static_cast<long long>(f->Cin) * P;
      g.sAm = W;
      g.sAk = 1;
      g.B = f->Fx;
      g.sBk = 2 * m;
      g.sBn = 1;
      g.C = f->Zb;
      g.sCb = static_cast<long long>(channels) * H * 2 * m;
      g.sCm = 2 * m;
      g.sCn = 1;
      g.M = channels * H;
      g.N = 2 * m;
      g.K = W;
      g.batch = batch;
      g.out_bf16 = 1;
      QLA_GEMM(g);
    }
    for (int part = 0; part < 2; ++part) {
      GemmDesc g;
      g.A = part ? f->A2 : f->A1;
      g.sAm = H;
      g.sAk = 1;
      g.B = f->Zb + part;
      g.sBb = static_cast<long long>(H) * 2 * m;
      g.sBk = 2 * m;
      g.sBn = 2;
      g.C = f->T[0];
      g.sCb = 4LL * m * m;
      g.sCm = m;
      g.sCn = 1;
      g.M = 4 * m;
      g.N = m;
      g.K = H;
      g.batch = batch * channels;
      g.beta = part;
      QLA_GEMM(g);
    }
  }
  QLA_HIP(hipMemsetAsync(f->band, 0, 2 * batch * sizeof(double), f->stream));
  hipLaunchKernelGGL(band_sums_kernel, dim3(64, batch), dim3(kBlock), 0, f->stream, f->T[0],
                     input + size_t(first_channel) * P, static_cast<long long>(f->Cin) * P,
                     channels, P, m, f->band);
  QLA_HIP(hipGetLastError());
  hipLaunchKernelGGL(band_final_kernel, dim3((batch + 63) / 64), dim3(64), 0, f->stream, f->band,
                     batch, double(H) * W, fraction_device);
  QLA_HIP(hipGetLastError());
  return QLA_OK;
}

qla_status qla_fno_output_energy(qla_fno* f, int batch, double* energy_device) {
  if (!f || !energy_device) return fail(QLA_EINVAL, "NULL argument");
  qla_status st = check_batch(f, batch);
  if (st != QLA_OK) return st;
  QLA_ON_DEVICE(f->device);
  QLA_HIP(hipMemsetAsync(energy_device, 0, batch * sizeof(double), f->stream));
  hipLaunchKernelGGL(energy_batch_kernel, dim3(256, batch), dim3(kBlock), 0, f->stream, f->out,
                     energy_device, size_t(f->Cout) * f->P);
  QLA_HIP(hipGetLastError());
  return QLA_OK;
}

qla_status qla_fno_pack(const double* q_device, const double* n_device, int nx, int ny,
                        double n_shift, uint16_t* input_device, uint16_t* target_device,
                        void* hip_stream) {
  if (!q_device || (input_device && !n_device) || nx < 1 || ny < 1)
    return fail(QLA_EINVAL, "bad pack arguments");
  const size_t P = size_t(nx) * ny;
  hipLaunchKernelGGL(pack_kernel, dim3(grid_for(P)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(hip_stream), q_device, n_device, P, n_shift,
                     input_device, target_device);
  QLA_HIP(hipGetLastError());
  return QLA_OK;
}

}  // extern "C"
