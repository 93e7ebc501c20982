// Batched, strided BF16 GEMM on the gfx950 matrix cores (v_mfma_f32_32x32x16_bf16),
// FP32 accumulation, used for every contraction of the neural-operator surrogate:
// channel mixing (1x1 convolutions), the truncated Fourier transforms written as
// products with cosine/sine bases, and all of their backward products.
//
//   C[b][m][n] = alpha * (sum_k A[b][m][k] B[b][k][n] + seg2)  (+ bias, res, C) (x GELU'(z))
//
// Every operand is addressed through its own strides, so transposed operands are
// just swapped strides. A block computes a 64x64 tile of C with 4 waves (2x2 of
// 32x32), stepping K by 32 through LDS tiles stored k-contiguous for both operands
// (one 16-byte LDS read per MFMA operand). The next K tile is fetched into registers
// while the current one is multiplied. Global loads take a 16-byte path when the
// operand is contiguous along k or along its free index, else an element path; all
// accesses are bounds-checked and out-of-range elements are zero.
//
// The optional second contraction (seg2) lets one launch add the inverse x transform
// of the spectral branch to the pointwise channel mixing of a Fourier layer (and the
// matching pair in the backward pass): its A operand is picked by the grid row of the
// output column and its B operand by the position within the row.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fno_internal.h"

namespace qla {
namespace fno {

namespace {

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// GELU and its derivative in the epilogues: the Abramowitz & Stegun 7.1.26 forms of
// fno_internal.h (with the library erff and expf they took most of the time of the
// epilogues that apply them to every element).
__device__ __forceinline__ float gelu(float x) { return gelu_as(x); }
__device__ __forceinline__ float gelu_prime(float x) { return gelu_prime_as(x); }

// One operand seen as rows r (A: m; B: n) by k: element (r, k) at p[r * sr + k * sk].
// Its access mode (a template argument where it is used) is 0 when k is contiguous,
// 1 when r is contiguous and 2 otherwise.
struct Operand {
  const uint16_t* p;
  long long sr, sk;
  int rmax, kmax;
};

int mode_of(long long sr, long long sk) { return sk == 1 ? 0 : (sr == 1 ? 1 : 2); }

__device__ __forceinline__ bool aligned16(const uint16_t* q) {
  return (reinterpret_cast<uintptr_t>(q) & 15) == 0;
}

// This thread's 8 elements of the 64 x 32 tile at (r0, k0).
template <int MODE>
__device__ __forceinline__ uint4 fetch(const Operand& o, int r0, int k0) {
  const int t = threadIdx.x;
  uint16_t v[8];
  if constexpr (MODE == 0) {
    const int r = r0 + (t >> 2), k = k0 + (t & 3) * 8;
    if (r < o.rmax && k + 8 <= o.kmax) {
      const uint16_t* q = o.p + r * o.sr + k;
      if (aligned16(q)) return *reinterpret_cast<const uint4*>(q);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
      v[i] = (r < o.rmax && k + i < o.kmax) ? o.p[r * o.sr + k + i] : uint16_t(0);
  } else if constexpr (MODE == 1) {
    const int k = k0 + (t >> 3), r = r0 + (t & 7) * 8;
    if (k < o.kmax && r + 8 <= o.rmax) {
      const uint16_t* q = o.p + k * o.sk + r;
      if (aligned16(q)) return *reinterpret_cast<const uint4*>(q);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
      v[i] = (k < o.kmax && r + i < o.rmax) ? o.p[k * o.sk + r + i] : uint16_t(0);
  } else {
    const int k = k0 + (t & 31);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = r0 + (t >> 5) + 8 * i;
      v[i] = (r < o.rmax && k < o.kmax) ? o.p[r * o.sr + k * o.sk] : uint16_t(0);
    }
  }
  uint4 w;
  __builtin_memcpy(&w, v, 16);
  return w;
}

// LDS tiles hold element (r, k) of an operand at lds[r][col(r, k)]: k-contiguous in
// groups of 8 (one 16-byte MFMA operand read), with the group index XORed by bits 3-4
// of the row. Rows are 16-byte aligned, so without the swizzle the transposing stores
// of row-contiguous operands (rows 8 apart in one instruction) all land in the same
// LDS banks.
__device__ __forceinline__ int col(int r, int k) {
  return ((((k >> 3) ^ (r >> 3)) & 3) << 3) | (k & 7);
}

// Stores fetched elements into the LDS tile.
template <int MODE>
__device__ __forceinline__ void stash(uint16_t (*lds)[kBK + kPad], uint4 w) {
  const int t = threadIdx.x;
  if constexpr (MODE == 0) {
    const int r = t >> 2;
    *reinterpret_cast<uint4*>(&lds[r][col(r, (t & 3) * 8)]) = w;
    return;
  }
  uint16_t v[8];
  __builtin_memcpy(v, &w, 16);
  if constexpr (MODE == 1) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = (t & 7) * 8 + i;
      lds[r][col(r, t >> 3)] = v[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = (t >> 5) + 8 * i;
      lds[r][col(r, t & 31)] = v[i];
    }
  }
}

// bias, residual, accumulate-into-C and GELU' factor of one output element
__device__ __forceinline__ float finish(const GemmDesc& g, float v, int b, int m, int n,
                                        long long co) {
  if (g.bias) v += g.bias[m];
  if (g.res) v += g.res[b * g.sRb + m * g.sRm + n * g.sRn];
  if (g.beta) {
    v += g.out_bf16 ? bf16_to_f32(static_cast<const uint16_t*>(g.C)[co])
                    : static_cast<const float*>(g.C)[co];
  }
  if (g.gz) v *= gelu_prime(bf16_to_f32(g.gz[co]));
  return v;
}

constexpr int kStageBytes = kBM * (kBN + 4) * 4;  // FP32 staging tile

// Writes this lane's 16 values (GELU of them if act) through LDS as 16-byte row chunks.
__device__ __forceinline__ void store_tile_bf16(const GemmDesc& g, uint16_t* dst,
                                                const float* val, bool act, int b, int m0,
                                                int n0, int nl, char* smem) {
  uint16_t(*st)[kBN + 8] = reinterpret_cast<uint16_t(*)[kBN + 8]>(smem);
  const int t = threadIdx.x, lane = t & 63, wm = (t >> 6) >> 1;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float v = val[4 * i + j];
      st[wm * 32 + 8 * i + 4 * (lane >> 5) + j][nl] = f32_to_bf16(act ? gelu(v) : v);
    }
  __syncthreads();
#pragma unroll
  for (int c = t; c < kBM * kBN / 8; c += 256) {
    const int r = c >> 3, cc = (c & 7) * 8, m = m0 + r, n = n0 + cc;
    if (m >= g.M) continue;
    uint16_t* q = dst + b * g.sCb + m * g.sCm + n;
    if (n + 8 <= g.N) {
      __builtin_nontemporal_store(*reinterpret_cast<const u32x4v*>(&st[r][cc]),
                                  reinterpret_cast<u32x4v*>(q));
    } else {
      for (int e = 0; e < 8 && n + e < g.N; ++e) q[e] = st[r][cc + e];
    }
  }
}

__device__ __forceinline__ void store_tile_f32(const GemmDesc& g, float* dst, const float* val,
                                               int b, int m0, int n0, int nl, char* smem) {
  float(*st)[kBN + 4] = reinterpret_cast<float(*)[kBN + 4]>(smem);
  const int t = threadIdx.x, lane = t & 63, wm = (t >> 6) >> 1;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) st[wm * 32 + 8 * i + 4 * (lane >> 5) + j][nl] = val[4 * i + j];
  __syncthreads();
#pragma unroll
  for (int c = t; c < kBM * kBN / 4; c += 256) {
    const int r = c >> 4, cc = (c & 15) * 4, m = m0 + r, n = n0 + cc;
    if (m >= g.M) continue;
    float* q = dst + b * g.sCb + m * g.sCm + n;
    if (n + 4 <= g.N) {
      __builtin_nontemporal_store(*reinterpret_cast<const f32x4v*>(&st[r][cc]),
                                  reinterpret_cast<f32x4v*>(q));
    } else {
      for (int e = 0; e < 4 && n + e < g.N; ++e) q[e] = st[r][cc + e];
    }
  }
}

// AM, BM: access modes of A and B; B2M: of the second contraction's B operand (its A
// operand is k-contiguous), or 3 when there is no second contraction.
template <int AM, int BM, int B2M>
__global__ __launch_bounds__(256) void gemm_kernel(GemmDesc g) {
  // LDS: the two operand tiles, later reused to stage the output tile
  __shared__ __attribute__((aligned(16))) char smem[kStageBytes];
  uint16_t(*As)[kBK + kPad] = reinterpret_cast<uint16_t(*)[kBK + kPad]>(smem);
  uint16_t(*Bs)[kBK + kPad] =
      reinterpret_cast<uint16_t(*)[kBK + kPad]>(smem + kBM * (kBK + kPad) * sizeof(uint16_t));
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN;
  const int z = blockIdx.z;
  const int b = z / g.ksplit, split = z % g.ksplit;
  const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + kBK - 1) / kBK * kBK;
  const int kb = min(g.K, split * kchunk), ke = min(g.K, kb + kchunk);
  // first contraction over [kb, ke): operands shifted so that k counts from kb
  const Operand a1{g.A + b * g.sAb + kb * g.sAk, g.sAm, g.sAk, g.M, ke - kb};
  const Operand b1{g.B + b * g.sBb + kb * g.sBk, g.sBn, g.sBk, g.N, ke - kb};
  const int s1 = ke > kb ? (ke - kb + kBK - 1) / kBK : 0;
  // second contraction: the tile's columns lie in one grid row y
  Operand a2{}, b2{};
  int s2 = 0;
  if constexpr (B2M != 3) {
    const int y = n0 / g.row, x0 = n0 % g.row;
    a2 = Operand{g.A2 + b * g.sA2b + y * g.sA2y, g.sA2m, 1, g.M, g.K2};
    b2 = Operand{g.B2 + x0 * g.sB2x, g.sB2x, g.sB2k, g.N - n0, g.K2};
    s2 = (g.K2 + kBK - 1) / kBK;
  }
  constexpr int kB2 = B2M == 3 ? 2 : B2M;
  const int steps = s1 + s2;
  const bool do_rowsum = g.rowsum != nullptr && blockIdx.y == 0;
  f32x16 acc = {};
  float rs = 0.f;
  uint4 ra = {}, rb = {};
  if (s1 > 0) {
    ra = fetch<AM>(a1, m0, 0);
    rb = fetch<BM>(b1, n0, 0);
  } else if constexpr (B2M != 3) {
    ra = fetch<0>(a2, m0, 0);
    rb = fetch<kB2>(b2, 0, 0);
  }
  for (int s = 0; s < steps; ++s) {
    const bool first = s < s1;
    if (B2M == 3 || first) {
      stash<AM>(As, ra);
      stash<BM>(Bs, rb);
    } else {
      stash<0>(As, ra);
      stash<kB2>(Bs, rb);
    }
    __syncthreads();
    if (s + 1 < steps) {
      if (B2M == 3 || s + 1 < s1) {
        ra = fetch<AM>(a1, m0, (s + 1) * kBK);
        rb = fetch<BM>(b1, n0, (s + 1) * kBK);
      } else {
        ra = fetch<0>(a2, m0, (s + 1 - s1) * kBK);
        rb = fetch<kB2>(b2, 0, (s + 1 - s1) * kBK);
      }
    }
    if (do_rowsum && first) {
      const uint16_t* row = &As[t >> 2][(t & 3) * 8];  // all groups of the row, any order
#pragma unroll
      for (int i = 0; i < 8; ++i) rs += bf16_to_f32(row[i]);
    }
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      const int ra = wm * 32 + (lane & 31), rb = wn * 32 + (lane & 31);
      const int kg = kk + 8 * (lane >> 5);
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[ra][col(ra, kg)]);
      const bf16x8 bb = *reinterpret_cast<const bf16x8*>(&Bs[rb][col(rb, kg)]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  if (do_rowsum) {
    // the 4 threads of a tile row are adjacent lanes
    rs += __shfl_xor(rs, 1);
    rs += __shfl_xor(rs, 2);
    const int m = m0 + (t >> 2);
    if ((t & 3) == 0 && m < g.M) atomicAdd(&g.rowsum[m], rs);
  }
  // epilogue: accumulator 4i + j holds row 8i + 4(lane/32) + j, column lane % 32
  if (!g.C && !g.act) return;
  const int nl = wn * 32 + (lane & 31), n = n0 + nl;
  if (!g.vec) {
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
        v = finish(g, v, b, m, n, co);
        if (g.C) {
          if (g.out_bf16) {
            static_cast<uint16_t*>(g.C)[co] = f32_to_bf16(v);
          } else {
            static_cast<float*>(g.C)[co] = v;
          }
        }
        if (g.act) g.act[co] = f32_to_bf16(gelu(v));
      }
    }
    return;
  }
  // vector epilogue (unit column stride, 16-byte aligned rows): finish the values in
  // registers, stage the tile in LDS and write each row with 16-byte non-temporal stores
  // (outputs are consumed by a later launch; measured faster for the consumers, e.g.
  // the narrow projection after projection 1: 249 -> 207 us)
  float val[16];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + wm * 32 + 8 * i + 4 * (lane >> 5) + j;
      float v = g.alpha * acc[4 * i + j];
      if (m < g.M && n < g.N) v = finish(g, v, b, m, n, b * g.sCb + m * g.sCm + n);
      val[4 * i + j] = v;
    }
  }
  if (g.C) {
    if (g.out_bf16) {
      store_tile_bf16(g, static_cast<uint16_t*>(g.C), val, false, b, m0, n0, nl, smem);
    } else {
      store_tile_f32(g, static_cast<float*>(g.C), val, b, m0, n0, nl, smem);
    }
  }
  if (g.act) store_tile_bf16(g, g.act, val, true, b, m0, n0, nl, smem);
}

}  // namespace

hipError_t launch_gemm(const GemmDesc& g, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.ksplit <= 0) return hipSuccess;
  if (g.K <= 0 && g.K2 <= 0) return hipSuccess;
  if (g.K2 > 0 && (g.row <= 0 || g.row % kBN != 0 || g.ksplit != 1 || g.atomic))
    return hipErrorInvalidValue;
  if (g.atomic && (g.bias || g.res || g.beta || g.gz || g.act || g.out_bf16 || !g.C))
    return hipErrorInvalidValue;
  if (g.beta && !g.C) return hipErrorInvalidValue;
  if (!g.C && !g.act && !g.rowsum) return hipErrorInvalidValue;
  if (g.K2 > 0 && g.sA2k != 1) return hipErrorInvalidValue;
  // M tiles along x (no practical limit), N tiles and batch x split along y and z
  const long long ny = (g.N + kBN - 1) / kBN, nz = static_cast<long long>(g.batch) * g.ksplit;
  if (ny > 65535 || nz > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((g.M + kBM - 1) / kBM, static_cast<unsigned>(ny), static_cast<unsigned>(nz));
  const int am = mode_of(g.sAm, g.sAk), bm = mode_of(g.sBn, g.sBk);
  const int b2m = g.K2 > 0 ? mode_of(g.sB2x, g.sB2k) : 3;
  if (b2m == 2) return hipErrorInvalidValue;
  using Kernel = void (*)(GemmDesc);
  static const Kernel table[3][3][3] = {
#define QLA_GEMM_ROW(a, b) {gemm_kernel<a, b, 0>, gemm_kernel<a, b, 1>, gemm_kernel<a, b, 3>}
      {QLA_GEMM_ROW(0, 0), QLA_GEMM_ROW(0, 1), QLA_GEMM_ROW(0, 2)},
      {QLA_GEMM_ROW(1, 0), QLA_GEMM_ROW(1, 1), QLA_GEMM_ROW(1, 2)},
      {QLA_GEMM_ROW(2, 0), QLA_GEMM_ROW(2, 1), QLA_GEMM_ROW(2, 2)},
#undef QLA_GEMM_ROW
  };
  const Kernel k = table[am][bm][b2m == 3 ? 2 : b2m];
  GemmDesc d = g;
  // 16-byte row stores need unit column stride and 16-byte aligned row starts
  const long long step = g.out_bf16 || !g.C ? 8 : 4;
  auto ok = [&](const void* p) {
    return !p || (reinterpret_cast<uintptr_t>(p) & 15) == 0;
  };
  d.vec = !g.atomic && g.sCn == 1 && g.sCm % step == 0 && g.sCb % step == 0 && ok(g.C) &&
          ok(g.act) && (!g.act || (g.sCm % 8 == 0 && g.sCb % 8 == 0));
  hipLaunchKernelGGL(k, grid, dim3(256), 0, stream, d);
  return hipGetLastError();
}

}  // namespace fno
}  // namespace qla
