// Device-side building blocks of the QLA step for gfx950: power series for the
// rotation coefficients, the three-shear form of a 2x2 rotation, and the
// wavefront-wide lane shifts used for neighbour exchange along x.
#pragma once

#include <hip/hip_runtime.h>

#include <array>

namespace qla {

// ---------------------------------------------------------------------------------
// Power-series coefficients, computed at compile time from their definitions:
//   sin x = x * sum_k S_k x^{2k},  S_k = (-1)^k / (2k+1)!
//   cos x =     sum_k K_k x^{2k},  K_k = (-1)^k / (2k)!
//   tan x = x * sum_k T_k x^{2k},  T_0 = 1, (2k+1) T_k = sum_{i+j=k-1} T_i T_j,
// the last from tan' = 1 + tan^2.
constexpr int kMaxTerms = 16;

constexpr std::array<double, kMaxTerms> make_sin_coeffs() {
  std::array<double, kMaxTerms> c{};
  double f = 1.0;  // (2k+1)!
  for (int k = 0; k < kMaxTerms; ++k) {
    if (k > 0) f *= double(2 * k) * double(2 * k + 1);
    c[k] = ((k & 1) ? -1.0 : 1.0) / f;
  }
  return c;
}

constexpr std::array<double, kMaxTerms> make_cos_coeffs() {
  std::array<double, kMaxTerms> c{};
  double f = 1.0;  // (2k)!
  for (int k = 0; k < kMaxTerms; ++k) {
    if (k > 0) f *= double(2 * k - 1) * double(2 * k);
    c[k] = ((k & 1) ? -1.0 : 1.0) / f;
  }
  return c;
}

constexpr std::array<double, kMaxTerms> make_tan_coeffs() {
  std::array<double, kMaxTerms> c{};
  c[0] = 1.0;
  for (int k = 1; k < kMaxTerms; ++k) {
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += c[i] * c[k - 1 - i];
    c[k] = acc / double(2 * k + 1);
  }
  return c;
}

constexpr std::array<double, kMaxTerms> kSinC = make_sin_coeffs();
constexpr std::array<double, kMaxTerms> kCosC = make_cos_coeffs();
constexpr std::array<double, kMaxTerms> kTanC = make_tan_coeffs();

// Number of series terms per precision and angle class, enough for the working
// precision when every series argument is within the class bound:
//   kSmall: |x| <= 1/8 (collision angles theta <= 1/16, potential half-angles
//           beta/2 <= 1/16; the default delta = 0.25 with n >= 1 is in this class);
//   kLarge: |x| <= 1   (theta <= 1/2, beta/2 <= 1/2).
// The host measures the largest angles when n is set and picks the class.
enum AngleClass : int { kSmall = 0, kLarge = 1 };

// ---------------------------------------------------------------------------------
// Two adjacent lattice columns held by one lane (FP32 stepping only). Every operation
// acts on the two columns alike, so each column goes through exactly the arithmetic
// of the one-column form and the results are bitwise the same; what changes is that a
// wavefront covers 128 columns, so its halo columns are a smaller share of the lanes,
// a lane shift moves one register for two columns, and every load or store moves
// 8 bytes per lane.
struct F32Pair {
  float x, y;
  F32Pair() = default;
  __device__ constexpr F32Pair(float a, float b) : x(a), y(b) {}
  __device__ explicit constexpr F32Pair(double v) : x(float(v)), y(float(v)) {}
  friend __device__ __forceinline__ F32Pair operator-(F32Pair a) { return {-a.x, -a.y}; }
  friend __device__ __forceinline__ F32Pair operator+(F32Pair a, F32Pair b) {
    return {a.x + b.x, a.y + b.y};
  }
  friend __device__ __forceinline__ F32Pair operator-(F32Pair a, F32Pair b) {
    return {a.x - b.x, a.y - b.y};
  }
  friend __device__ __forceinline__ F32Pair operator*(F32Pair a, F32Pair b) {
    return {a.x * b.x, a.y * b.y};
  }
  friend __device__ __forceinline__ F32Pair operator*(float a, F32Pair b) {
    return {a * b.x, a * b.y};
  }
  friend __device__ __forceinline__ F32Pair fma(F32Pair a, F32Pair b, F32Pair c) {
    return {fmaf(a.x, b.x, c.x), fmaf(a.y, b.y, c.y)};
  }
};

template <typename T, int C> struct Terms;
template <> struct Terms<double, kSmall> { static constexpr int kSin = 6, kTan = 6, kCos = 7; };
template <> struct Terms<double, kLarge> { static constexpr int kSin = 10, kTan = 13, kCos = 11; };
template <> struct Terms<float, kSmall> { static constexpr int kSin = 3, kTan = 3, kCos = 3; };
template <> struct Terms<float, kLarge> { static constexpr int kSin = 6, kTan = 7, kCos = 7; };
template <int C> struct Terms<F32Pair, C> : Terms<float, C> {};

template <typename T, int N>
__device__ __forceinline__ T odd_series(T x, const std::array<double, kMaxTerms>& c) {
  const T x2 = x * x;
  T acc = T(c[N - 1]);
#pragma unroll
  for (int k = N - 2; k >= 0; --k) acc = fma(acc, x2, T(c[k]));
  return x * acc;
}

template <typename T, int N>
__device__ __forceinline__ T even_series(T x, const std::array<double, kMaxTerms>& c) {
  const T x2 = x * x;
  T acc = T(c[N - 1]);
#pragma unroll
  for (int k = N - 2; k >= 0; --k) acc = fma(acc, x2, T(c[k]));
  return acc;
}

template <typename T, int C> __device__ __forceinline__ T sin_series(T x) {
  return odd_series<T, Terms<T, C>::kSin>(x, kSinC);
}
template <typename T, int C> __device__ __forceinline__ T cos_series(T x) {
  return even_series<T, Terms<T, C>::kCos>(x, kCosC);
}
template <typename T, int C> __device__ __forceinline__ T tan_series(T x) {
  return odd_series<T, Terms<T, C>::kTan>(x, kTanC);
}

// 1/n: hardware reciprocal estimate refined by Newton steps to the working precision.
__device__ __forceinline__ double recip(double v) {
  double r = __builtin_amdgcn_rcp(v);
  double e = fma(-v, r, 1.0);
  r = fma(r, e, r);
  e = fma(-v, r, 1.0);
  r = fma(r, e, r);
  e = fma(-v, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float v) {
  float r = __builtin_amdgcn_rcpf(v);
  const float e = fmaf(-v, r, 1.0f);
  return fmaf(r, e, r);
}
__device__ __forceinline__ F32Pair recip(F32Pair v) { return {recip(v.x), recip(v.y)}; }

// ---------------------------------------------------------------------------------
// A rotation R(phi): a' = cos(phi) a - sin(phi) p, p' = sin(phi) a + cos(phi) p,
// applied as three shears with t = tan(phi/2), s = sin(phi):
//   a <- a - t p;  p <- p + s a;  a <- a - t p.
// Exact in real arithmetic; with rounded (t, s) each shear still has determinant
// exactly 1, so long runs show no systematic growth or decay of |a|^2 + |p|^2
// (rounded cos/sin pairs would scale the norm by sqrt(c^2 + s^2) every time).
// R(-phi) uses (-t, -s).
template <typename T> struct Shear {
  T t, s;
};

template <typename T, int C>
__device__ __forceinline__ Shear<T> shear_of(T phi) {
  return {tan_series<T, C>(T(0.5) * phi), sin_series<T, C>(phi)};
}

template <typename T>
__device__ __forceinline__ void rotate(T& a, T& p, T t, T s) {
  a = fma(-t, p, a);
  p = fma(s, a, p);
  a = fma(-t, p, a);
}

// The first output a' of R(phi) on (a, p), when p' is produced elsewhere.
template <typename T>
__device__ __forceinline__ T rotate_first(T a, T p, T t, T s) {
  const T a1 = fma(-t, p, a);
  const T p1 = fma(s, a1, p);
  return fma(-t, p1, a1);
}

// The second output p' of R(phi) on (a, p), when a' is produced elsewhere. It
// repeats the first shear bit for bit, so both halves of a pair held by two
// lanes see the same intermediate value.
template <typename T>
__device__ __forceinline__ T rotate_second(T a, T p, T t, T s) {
  const T a1 = fma(-t, p, a);
  return fma(s, a1, p);
}

// ---------------------------------------------------------------------------------
// Wavefront-wide lane shifts (DPP wave_shr:1 / wave_shl:1 on the 64-lane wave):
// from_left(v) in lane l is v of lane l-1, from_right(v) is v of lane l+1; the end
// lanes receive 0 (they are halo lanes whose results are never stored).
__device__ __forceinline__ int dpp_from_left(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_from_right(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);
}

__device__ __forceinline__ float from_left(float v) {
  return __builtin_bit_cast(float, dpp_from_left(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float from_right(float v) {
  return __builtin_bit_cast(float, dpp_from_right(__builtin_bit_cast(int, v)));
}
// A lane holding columns (2l, 2l+1): the left neighbour of column 2l is column 2l-1,
// the second of lane l-1; the right neighbour of column 2l+1 is the first of lane l+1.
__device__ __forceinline__ F32Pair from_left(F32Pair v) { return {from_left(v.y), v.x}; }
__device__ __forceinline__ F32Pair from_right(F32Pair v) { return {v.y, from_right(v.x)}; }
__device__ __forceinline__ double from_left(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_from_left(int(b));
  const int hi = dpp_from_left(int(b >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) |
                                        static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double from_right(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_from_right(int(b));
  const int hi = dpp_from_right(int(b >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) |
                                        static_cast<unsigned int>(lo));
}

// ---------------------------------------------------------------------------------
// Blocks of one launch are dealt round-robin to the 8 XCDs (each with its own L2).
// Renumber them so that every XCD works on one contiguous range of tiles, which
// keeps neighbouring tiles (and the halo rows they share) in the same L2.
__device__ __forceinline__ int xcd_contiguous_block(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

}  // namespace qla
