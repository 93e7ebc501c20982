// Fused QLA time step for the E_z triple (q2, q3, q4) = (n Ez, Bx, By) on gfx950.
//
// One launch applies one full step of Eq. (2e14), Q <- V_y V_x U_y U_x Q, reading
// each amplitude plane and n once from HBM and writing each amplitude plane once.
//
// Operator algebra. Every set of four factors in U_x (Eq. 2e6) has the form
// "stream, collide, stream back, collide" on one pair. Pushing the two shifts
// through the collision between them turns each set into two rotations that
// move no data: a rotation of every on-site pair (a_i, p_i), then a rotation of
// the neighbouring pairs (a_i, p_{i-1}) or (a_i, p_{i+1}). With a = q2 and p = q4
// (x) or p = q3 (y), applied first to last:
//   set 1: C^T(th_i) on (a_i, p_i);  C(th_i)       on (a_i, p_{i-1})
//   set 2: C^T(th_i) on (a_i, p_i);  C(th_{i-1})   on (a_i, p_{i-1})
//   set 3: C(th_i)   on (a_i, p_i);  C^T(th_i)     on (a_i, p_{i+1})
//   set 4: C(th_i)   on (a_i, p_i);  C^T(th_{i+1}) on (a_i, p_{i+1})
// where C is the 2x2 block of C_x (Eq. 2e3) on (q2, q4), a rotation R(+th), or of
// C_y (Eq. 2e8) on (q2, q3), a rotation R(-th); th = delta / (4 n) (Eq. 2e4). U_y
// (Eq. 2e9) is the same along y. Each output depends on inputs at most 4 sites
// away along the operator's axis.
//
// Potentials (Eqs. 2e11-2e13), beta = delta^2 (dn/dx) / n^2 with centred
// differences, i.e. beta/2 = (delta/4) (n_{+1} - n_{-1}) / n^2 in cell units:
//   SKEW_HALF: V_x = R(-beta_x/2) on (q2, q4); V_y = R(+beta_y/2) on (q2, q3).
//   PAPER:     q4 <- -sin(beta_x) q2 + cos(beta_x) q4; q3 <- sin(beta_y) q2 + cos(beta_y) q3.
//   BSTREAM:   no potentials; sets 2 and 4 of U_x and U_y are replaced by copies of
//              sets 1 and 3 (every set streams the B-qubit p), so every neighbour
//              pair takes the angle of its a site (a scheme beyond the paper).
//
// The B_z triple (q0, q1, q5) follows the same algebra with a = q5 (streamed by S_25
// along both axes), p = q1 along x (streamed by S_14) and p = q0 along y (by S_03):
// on these pairs C_x is R(-th) and C_y is R(+th), the E_z rotations with th negated,
// and the SKEW_HALF potentials are the same rotations as above. The sign of th comes
// with the launch arguments; the planes are passed as (a, p_y, p_x).
//
// Mapping to the machine. A wavefront owns a strip of output columns and a segment
// of output rows. Its 64 lanes hold consecutive columns, one per lane (or, in FP32
// on lattices of even width, two per lane: 128 columns), with 4 halo columns per
// step each side (periodic wrap). The wave marches down the rows:
//   - each incoming row gets U_x across the lanes, with the neighbour values
//     taken by DPP lane shifts (no LDS, no barriers);
//   - U_y runs down the rows inside each lane as a software pipeline: when row r
//     arrives, set 1 finishes row r-1, set 2 row r-2, set 3 row r-3 and set 4 row
//     r-4, which then gets V_x, V_y and is stored.
// The rows of the window live in registers, indexed modulo the window depth with
// the loop unrolled that many times so every index is static; loads run 2-3 rows
// ahead. The segment starts 4 rows early and ends 4 rows late (vertical halo).
// One pass can also apply two steps (temporal blocking, see Marcher). Rotations use the
// three-shear form (qla_device.h); angles come from n on the fly, so HBM traffic
// is exactly three amplitude planes in and out plus n in.
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>
#include <utility>

#include "qla_device.h"
#include "qla_internal.h"

namespace qla {

namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
// A buffer store whose offset is at least the buffer's size is discarded by the
// hardware; stores of halo lanes and of rows outside the segment use this offset
// instead of a branch, so the memory counters stay static for the compiler.
constexpr unsigned kDropOffset = 0x80000000u;
// Largest plane one buffer descriptor addresses with these offsets (and below which
// kDropOffset is out of range).
constexpr size_t kMaxPlaneDescriptorBytes = size_t(1) << 31;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* p, unsigned bytes) {
  // raw buffer (stride 0), 32-bit dwords, range-checked against `bytes`
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes),
                                           0x00020000);
}

__device__ __forceinline__ unsigned long long bits_of(double v) {
  return __builtin_bit_cast(unsigned long long, v);
}
__device__ __forceinline__ unsigned long long bits_of(float v) {
  return __builtin_bit_cast(unsigned int, v);
}
// The bit pattern of lane 0's value, in scalar registers.
__device__ __forceinline__ unsigned long long lane0_bits(double v) {
  const unsigned long long b = bits_of(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(b));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(b >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}
__device__ __forceinline__ unsigned long long lane0_bits(float v) {
  return __builtin_amdgcn_readfirstlane(__builtin_bit_cast(unsigned, v));
}
__device__ __forceinline__ unsigned long long lane0_bits(F32Pair v) { return lane0_bits(v.x); }
// Does this lane hold a value other than the bit pattern b?
template <typename V>
__device__ __forceinline__ bool differs(V v, unsigned long long b) {
  return bits_of(v) != b;
}
template <>
__device__ __forceinline__ bool differs(F32Pair v, unsigned long long b) {
  return (bits_of(v.x) != b) | (bits_of(v.y) != b);
}

// The value a lane holds: one column of T, or two FP32 columns.
template <typename T, int CPL> struct LaneOf { using type = T; };
template <> struct LaneOf<float, 2> { using type = F32Pair; };

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
}

// Cache policy of the amplitude stores. A single lattice's pass writes state that is
// next read by the following pass, long after it has left the caches, while the rows
// the pass loads are re-read by neighbouring tiles (halo rows and columns): its stores
// are non-temporal (the NT bit of gfx94x/gfx950 buffer instructions), measured 1-4%
// faster on 4096^2-16384^2 lattices and even on 1024^2-3072^2. The batched kernel
// measured 12% slower with them, so its stores keep the default policy.
constexpr int kStoreNonTemporal = 2;
constexpr int kStoreDefault = 0;

template <typename T, int SP = kStoreDefault>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
  if constexpr (sizeof(T) == 8) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, SP);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, SP);
  }
}

template <typename T>
struct StepArgs {
  const T* q2i;
  const T* q3i;
  const T* q4i;
  const T* n;
  T* q2o;
  T* q3o;
  T* q4o;
  unsigned plane_bytes;  // pitch * ny * sizeof(T) (planes of at most 2^31 bytes), else 0
  int nx, ny, pitch, strips, segs, rows_per_seg, iters;  // pitch: row pitch in elements
  T d4;  // delta / 4
  T dc;  // collision angle over 1/n: +delta/4 (E_z triple) or -delta/4 (B_z triple)
};

// kWin: register window depth in rows (the loop is unrolled kWin times so every
// window index is static); PF: how many rows ahead the loads run; TS: how many
// steps one pass applies (temporal blocking).
//
// With TS steps per pass, stage k (k = 0 .. TS-1) applies step k + 1. Stage 0
// receives the freshly loaded row r; stage k receives row r - 4k, the row stage
// k-1 completed in the same iteration, and completes row r - 4k - 4. The stages
// share one window: a row keeps its slot from its load until its store. Each
// stage widens the dependence by 4 cells in x and y, so a pass has 4 TS halo
// columns on each side of the strip and 4 TS halo rows at each end of a segment.
// Plane addressing: one buffer descriptor per plane, offsets within it (planes of at
// most 2^31 bytes), or a descriptor per row, based at the row's 64-bit address in
// scalar registers (any plane size; the offsets stay within one row).
enum Addressing : int { kPlaneDescriptors = 0, kRowDescriptors = 1 };

template <typename T, int VMODE, int CLS, int kWin, int PF, int TS, int CPL, int SP, int AM>
struct Marcher {
  static_assert(PF + 4 * TS + 2 <= kWin, "a prefetched row must not overwrite a live one");
  using V = typename LaneOf<T, CPL>::type;
  static_assert(sizeof(V) == CPL * sizeof(T), "one or two columns per lane");
  // B streaming: every set streams the B-qubit, so each neighbour pair takes the angle
  // of its a site, and there are no potentials
  static constexpr bool kBStream = VMODE == kVBStream;
  // FP32 (one or two columns per lane): neighbour pairs of U_x split between lanes
  static constexpr bool kSplitPairs = sizeof(T) == 4;
  // Row window: amplitudes, index, 1/n and the collision shear of each row.
  V A[kWin], P4[kWin], P3[kWin], N[kWin], M[kWin], Tt[kWin], Ts[kWin];
  // Per-row wave-uniform facts, one bit per slot in scalar registers: umask bit s
  // says all 64 lanes of the row in slot s hold the same n; emask bit s says so
  // and that this n equals the previous row's (also uniform) n. In a uniform row
  // the neighbours' collision angles equal the lane's own; where a row and its
  // two vertical neighbours hold one common n every potential angle is exactly 0
  // (V = I).
  unsigned umask, emask;
  unsigned long long nb_prev;  // n's bit pattern in lane 0 of the previous row
  __amdgpu_buffer_rsrc_t r2i, r3i, r4i, rn, r2o, r3o, r4o;  // kPlaneDescriptors
  const char *b2i, *b3i, *b4i, *bn;                          // kRowDescriptors: plane bases
  char *b2o, *b3o, *b4o;
  unsigned col_bytes;    // this lane's (first) column (wrapped) in bytes
  unsigned store_bytes;  // col_bytes for lanes that own an output column, else kDropOffset
  unsigned row_bytes;    // pitch * sizeof(T)
  int yin;               // row index of the next row to load (wrapped)

  static constexpr int slot(int s, int back) { return ((s - back) % kWin + kWin) % kWin; }

  // y is uniform across the wave: the row offset is a scalar register and every
  // lane adds its fixed column offset.
  __device__ __forceinline__ void load_row(int s, int y) {
    const unsigned yu = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(y));
    if constexpr (AM == kRowDescriptors) {
      const size_t off = static_cast<size_t>(yu) * row_bytes;
      A[s] = buf_load<V>(plane_rsrc(b2i + off, row_bytes), col_bytes, 0u);
      P3[s] = buf_load<V>(plane_rsrc(b3i + off, row_bytes), col_bytes, 0u);
      P4[s] = buf_load<V>(plane_rsrc(b4i + off, row_bytes), col_bytes, 0u);
      N[s] = buf_load<V>(plane_rsrc(bn + off, row_bytes), col_bytes, 0u);
    } else {
      const unsigned soff = yu * row_bytes;
      A[s] = buf_load<V>(r2i, col_bytes, soff);
      P3[s] = buf_load<V>(r3i, col_bytes, soff);
      P4[s] = buf_load<V>(r4i, col_bytes, soff);
      N[s] = buf_load<V>(rn, col_bytes, soff);
    }
  }

  // Stores of one output row (discarded for voff = kDropOffset).
  __device__ __forceinline__ void store_row(int s, unsigned yo, unsigned voff) {
    if constexpr (AM == kRowDescriptors) {
      const size_t off = static_cast<size_t>(yo) * row_bytes;
      buf_store<V, SP>(A[s], plane_rsrc(b2o + off, row_bytes), voff, 0u);
      buf_store<V, SP>(P3[s], plane_rsrc(b3o + off, row_bytes), voff, 0u);
      buf_store<V, SP>(P4[s], plane_rsrc(b4o + off, row_bytes), voff, 0u);
    } else {
      const unsigned soff = yo * row_bytes;
      buf_store<V, SP>(A[s], r2o, voff, soff);
      buf_store<V, SP>(P3[s], r3o, voff, soff);
      buf_store<V, SP>(P4[s], r4o, voff, soff);
    }
  }

  // U_x on one row (slot s): lanes exchange neighbour values by DPP. In a
  // uniform row the neighbours' shears are the lane's own, and the FP64 form skips
  // their exchange (the two versions differ only in the end lanes, which are halo).
  __device__ __forceinline__ void ux(int s) {
    if constexpr (kSplitPairs) {
      // One lane shift per neighbour value, in every row: a branch on uniform rows
      // costs more here (its join copies and the negations it keeps from folding
      // into the FMAs) than the four shifts it would save.
      ux_with(s, from_left(Tt[s]), from_left(Ts[s]), from_right(Tt[s]), from_right(Ts[s]));
    } else if (umask & (1u << s)) {
      ux_with(s, Tt[s], Ts[s], Tt[s], Ts[s]);
    } else {
      ux_with(s, from_left(Tt[s]), from_left(Ts[s]), from_right(Tt[s]), from_right(Ts[s]));
    }
  }

  // The neighbour rotation of U_x on pair (a_i, p_j), j = i - 1 (kLeft) or i + 1,
  // split between the two lanes holding it: lane i forms a1 = a_i - t p_j, lane j
  // forms p_j' = p_j + s a1 from that a1, lane i forms a_i' = a1 - t p_j' from that
  // p_j'. These are the values rotate_first and rotate_second give (they form a1 in
  // both lanes), with three lane shifts instead of two and two FMAs fewer per pair:
  // the form used where a lane shift is one instruction (FP32). ta: the t that the
  // a-lane applies; sp: the s that the p-lane applies.
  template <bool kLeft>
  __device__ __forceinline__ void split_pair(V& a, V& p, V ta, V sp) {
    if constexpr (kLeft) {
      const V a1 = fma(-ta, from_left(p), a);
      p = fma(sp, from_right(a1), p);
      a = fma(-ta, from_left(p), a1);
    } else {
      const V a1 = fma(-ta, from_right(p), a);
      p = fma(sp, from_left(a1), p);
      a = fma(-ta, from_right(p), a1);
    }
  }

  __device__ __forceinline__ void ux_with(int s, V tl, V sl, V tr, V sr) {
    V a = A[s], p = P4[s];
    const V t0 = Tt[s], s0 = Ts[s];
    if constexpr (kSplitPairs) {
      // the sets below, with each neighbour pair split between its lanes
      rotate(a, p, -t0, -s0);
      split_pair<true>(a, p, t0, sr);
      rotate(a, p, -t0, -s0);
      if constexpr (kBStream) {
        split_pair<true>(a, p, t0, sr);
      } else {
        split_pair<true>(a, p, tl, s0);
      }
      rotate(a, p, t0, s0);
      split_pair<false>(a, p, -t0, -sl);
      rotate(a, p, t0, s0);
      if constexpr (kBStream) {
        split_pair<false>(a, p, -t0, -sl);
      } else {
        split_pair<false>(a, p, -tr, -s0);
      }
      A[s] = a;
      P4[s] = p;
      return;
    }
    // set 1: C^T on site; C(th_i) on (a_i, p_{i-1})
    rotate(a, p, -t0, -s0);
    {
      const V pm = from_left(p), ap = from_right(a);
      const V an = rotate_first(a, pm, t0, s0);
      p = rotate_second(ap, p, tr, sr);
      a = an;
    }
    // set 2: C^T on site; C(th_{i-1}) on (a_i, p_{i-1}); with B streaming a copy of
    // set 1 (the pair takes the angle of its a site)
    rotate(a, p, -t0, -s0);
    {
      const V pm = from_left(p), ap = from_right(a);
      const V an = kBStream ? rotate_first(a, pm, t0, s0) : rotate_first(a, pm, tl, sl);
      p = kBStream ? rotate_second(ap, p, tr, sr) : rotate_second(ap, p, t0, s0);
      a = an;
    }
    // set 3: C on site; C^T(th_i) on (a_i, p_{i+1})
    rotate(a, p, t0, s0);
    {
      const V pp = from_right(p), am = from_left(a);
      const V an = rotate_first(a, pp, -t0, -s0);
      p = rotate_second(am, p, -tl, -sl);
      a = an;
    }
    // set 4: C on site; C^T(th_{i+1}) on (a_i, p_{i+1}); with B streaming a copy of
    // set 3
    rotate(a, p, t0, s0);
    {
      const V pp = from_right(p), am = from_left(a);
      const V an = kBStream ? rotate_first(a, pp, -t0, -s0) : rotate_first(a, pp, -tr, -sr);
      p = kBStream ? rotate_second(am, p, -tl, -sl) : rotate_second(am, p, -t0, -s0);
      a = an;
    }
    A[s] = a;
    P4[s] = p;
  }

  // U_y pipeline of one stage after its row a (slot SA) arrived; C_y = R(-th),
  // C_y^T = R(+th).
  template <int SA>
  __device__ __forceinline__ void uy() {
    constexpr int s0 = SA, s1 = slot(SA, 1), s2 = slot(SA, 2), s3 = slot(SA, 3),
                  s4 = slot(SA, 4);
    // set 1 on row a: on-site C_y^T, then (a_a, p_{a-1}) with C_y(th_a)
    rotate(A[s0], P3[s0], Tt[s0], Ts[s0]);
    rotate(A[s0], P3[s1], -Tt[s0], -Ts[s0]);
    // set 2 on row a-1: on-site C_y^T, then (a_{a-1}, p_{a-2}) with C_y(th_{a-2})
    // (with B streaming: th_{a-1}, a copy of set 1)
    constexpr int s2a = kBStream ? s1 : s2;
    rotate(A[s1], P3[s1], Tt[s1], Ts[s1]);
    rotate(A[s1], P3[s2], -Tt[s2a], -Ts[s2a]);
    // set 3 on row a-2: on-site C_y, then (a_{a-3}, p_{a-2}) with C_y^T(th_{a-3})
    rotate(A[s2], P3[s2], -Tt[s2], -Ts[s2]);
    rotate(A[s3], P3[s2], Tt[s3], Ts[s3]);
    // set 4 on row a-3: on-site C_y, then (a_{a-4}, p_{a-3}) with C_y^T(th_{a-3})
    // (with B streaming: th_{a-4}, a copy of set 3)
    constexpr int s4a = kBStream ? s4 : s3;
    rotate(A[s3], P3[s3], -Tt[s3], -Ts[s3]);
    rotate(A[s4], P3[s3], Tt[s4a], Ts[s4a]);
  }

  // V_x, V_y on the row a - 4 that the stage just completed (slot SC).
  template <int SC>
  __device__ __forceinline__ void potentials(T d4) {
    if constexpr (VMODE == kVNone || VMODE == kVBStream) {
      return;
    } else {
      constexpr int sc = SC, sup = slot(SC, -1), sdn = slot(SC, 1);
      if ((emask & (1u << sc)) && (emask & (1u << sup))) return;
      const V m = M[sc];
      const V dm = d4 * m * m;
      const V nl = from_left(N[sc]), nr = from_right(N[sc]);
      const V hbx = (nr - nl) * dm;          // beta_x / 2
      const V hby = (N[sup] - N[sdn]) * dm;  // beta_y / 2
      if constexpr (VMODE == kVSkewHalf) {
        const Shear<V> vx = shear_of<V, CLS>(hbx);
        rotate(A[sc], P4[sc], -vx.t, -vx.s);
        const Shear<V> vy = shear_of<V, CLS>(hby);
        rotate(A[sc], P3[sc], vy.t, vy.s);
      } else {
        const V bx = hbx + hbx, by = hby + hby;
        const V sbx = sin_series<V, CLS>(bx), cbx = cos_series<V, CLS>(bx);
        P4[sc] = fma(-sbx, A[sc], cbx * P4[sc]);
        const V sby = sin_series<V, CLS>(by), cby = cos_series<V, CLS>(by);
        P3[sc] = fma(sby, A[sc], cby * P3[sc]);
      }
    }
  }

  template <int S0, int K>
  __device__ __forceinline__ void stage(T d4) {
    constexpr int sa = slot(S0, 4 * K);  // row arriving at this stage
    ux(sa);
    uy<sa>();
    potentials<slot(sa, 4)>(d4);
  }

  template <int S0>
  __device__ __forceinline__ void iteration(const StepArgs<T>& g, int r, int y0, int yend) {
    constexpr int sp = slot(S0, -PF), sout = slot(S0, 4 * TS);
    // loads for row r + PF (the slot held row r + PF - kWin, no longer needed).
    // Issued unconditionally, also past the segment's end (rows wrap, so they stay
    // in bounds): a branch here would make the compiler wait for them at once.
    load_row(sp, yin);
    yin = (yin + 1 == g.ny) ? 0 : yin + 1;
    // Is row r uniform? Then, if row r - 1 was uniform with the same n, its
    // collision shear and 1/n are reused; otherwise they are computed.
    constexpr int sprev = slot(S0, 1);
    const unsigned long long nb = lane0_bits(N[S0]);
    const bool uni = __builtin_amdgcn_ballot_w64(differs(N[S0], nb)) == 0;
    const bool same = uni && (umask & (1u << sprev)) && nb == nb_prev;
    umask = (umask & ~(1u << S0)) | (uni ? 1u << S0 : 0u);
    emask = (emask & ~(1u << S0)) | (same ? 1u << S0 : 0u);
    nb_prev = nb;
    if (same) {
      M[S0] = M[sprev];
      Tt[S0] = Tt[sprev];
      Ts[S0] = Ts[sprev];
    } else {
      const V m = recip(N[S0]);
      M[S0] = m;
      const Shear<V> c = shear_of<V, CLS>(g.dc * m);
      Tt[S0] = c.t;
      Ts[S0] = c.s;
    }
    [&]<int... K>(std::integer_sequence<int, K...>) {
      (stage<S0, K>(g.d4), ...);
    }(std::make_integer_sequence<int, TS>{});
    // row r - 4 TS has had all TS steps: output row y0 + r - 8 TS
    const int yo = y0 + r - 8 * TS;
    const bool row_ok = yo >= y0 && yo < yend;
    store_row(sout, row_ok ? static_cast<unsigned>(yo) : 0u, row_ok ? store_bytes : kDropOffset);
  }
};

// One wavefront's work: the tile (strip, seg) of one pass over the lattice of g. With
// two columns per lane the width is even (checked on the host), so a lane's pair
// (col, col + 1) never straddles the periodic wrap and lies wholly inside or outside
// the strip's output columns.
template <typename T, int VMODE, int CLS, int kWin, int PF, int TS, int CPL, int SP, int AM>
__device__ __forceinline__ void march(const StepArgs<T>& g, int strip, int seg, int lane) {
  constexpr int halo = 4 * TS;
  constexpr int strip_cols = kWave * CPL - 2 * halo;
  Marcher<T, VMODE, CLS, kWin, PF, TS, CPL, SP, AM> w;
  using V = typename Marcher<T, VMODE, CLS, kWin, PF, TS, CPL, SP, AM>::V;
  const int x0 = strip * strip_cols;
  const int c = CPL * lane - halo;  // the lane's first column, relative to the strip
  int col = (x0 + c) % g.nx;
  if (col < 0) col += g.nx;
  const bool store_lane = c >= 0 && c < strip_cols && x0 + c < g.nx;
  w.col_bytes = static_cast<unsigned>(col) * sizeof(T);
  w.store_bytes = store_lane ? w.col_bytes : kDropOffset;
  w.row_bytes = static_cast<unsigned>(g.pitch) * sizeof(T);
  if constexpr (AM == kRowDescriptors) {
    w.b2i = reinterpret_cast<const char*>(g.q2i);
    w.b3i = reinterpret_cast<const char*>(g.q3i);
    w.b4i = reinterpret_cast<const char*>(g.q4i);
    w.bn = reinterpret_cast<const char*>(g.n);
    w.b2o = reinterpret_cast<char*>(g.q2o);
    w.b3o = reinterpret_cast<char*>(g.q3o);
    w.b4o = reinterpret_cast<char*>(g.q4o);
  } else {
    w.r2i = plane_rsrc(g.q2i, g.plane_bytes);
    w.r3i = plane_rsrc(g.q3i, g.plane_bytes);
    w.r4i = plane_rsrc(g.q4i, g.plane_bytes);
    w.rn = plane_rsrc(g.n, g.plane_bytes);
    w.r2o = plane_rsrc(g.q2o, g.plane_bytes);
    w.r3o = plane_rsrc(g.q3o, g.plane_bytes);
    w.r4o = plane_rsrc(g.q4o, g.plane_bytes);
  }
  const int y0 = seg * g.rows_per_seg;
  const int yend = min(y0 + g.rows_per_seg, g.ny);
#pragma unroll
  for (int k = 0; k < kWin; ++k) {
    w.A[k] = w.P4[k] = w.P3[k] = w.N[k] = w.M[k] = w.Tt[k] = w.Ts[k] = V(T(0));
  }
  w.umask = 0;
  w.emask = 0;
  w.nb_prev = 0;
  int y = (y0 - halo) % g.ny;
  if (y < 0) y += g.ny;
  // The prologue issues the first PF rows in the same pattern as the loop body
  // (4 loads, then 3 stores, here discarded ones), so the compiler sees the same
  // outstanding memory operations on entry as on the back edge and keeps its
  // waits at the prefetch distance instead of draining the queue every trip.
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    w.load_row(k, y);
    y = (y + 1 == g.ny) ? 0 : y + 1;
    w.store_row(0, 0u, kDropOffset);
  }
  w.yin = y;

  for (int r = 0; r < g.iters; r += kWin) {
    [&]<int... K>(std::integer_sequence<int, K...>) {
      (w.template iteration<K>(g, r + K, y0, yend), ...);
    }(std::make_integer_sequence<int, kWin>{});
  }
}

template <typename T, int VMODE, int CLS, int kWin, int PF, int TS, int CPL, int AM>
__global__ __launch_bounds__(kWave * kWavesPerBlock) void qla_step_ez_kernel(StepArgs<T> g) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = threadIdx.x / kWave;
  const int blk = xcd_contiguous_block(blockIdx.x, gridDim.x);
  const int blocks_per_seg = (g.strips + kWavesPerBlock - 1) / kWavesPerBlock;
  const int seg = blk / blocks_per_seg;
  const int strip = (blk % blocks_per_seg) * kWavesPerBlock + wib;
  if (seg >= g.segs || strip >= g.strips) return;  // whole wave exits together
  march<T, VMODE, CLS, kWin, PF, TS, CPL, kStoreNonTemporal, AM>(g, strip, seg, lane);
}

// Batched passes. `args` holds two entries per instance (parity 0: the buffer that
// was current when the tables were built -> the other buffer; parity 1: back); pass p
// of instance i uses parity (p + parity[i]) & 1, where parity[i] records whether a
// previous run left instance i's buffers swapped. `items` lists (instance << 20 | tile)
// for all instances, ordered by decreasing pass count, so the items of the
// instances still running at pass p are the first counts[p] entries. The launch
// runs pass p; each wave strides over its items (the grid is sized to what stays
// resident, so the waves persist across items).
template <typename T, int VMODE, int CLS, int kWin, int PF, int TS>
__global__ __launch_bounds__(kWave * kWavesPerBlock) void qla_batch_kernel(
    const StepArgs<T>* __restrict__ args, const unsigned* __restrict__ items,
    const int* __restrict__ counts, const int* __restrict__ parity, int p) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = blockIdx.x * kWavesPerBlock + static_cast<int>(threadIdx.x / kWave);
  const int waves = gridDim.x * kWavesPerBlock;
  const int count = counts[p];
  for (int it = wave; it < count; it += waves) {
    const unsigned code = __builtin_amdgcn_readfirstlane(items[it]);
    const int inst = static_cast<int>(code >> 20);
    const int tile = static_cast<int>(code & 0xFFFFFu);
    const int par = __builtin_amdgcn_readfirstlane(parity[inst]);
    const StepArgs<T> g = args[2 * inst + ((p + par) & 1)];
    march<T, VMODE, CLS, kWin, PF, TS, 1, kStoreDefault, kPlaneDescriptors>(
        g, tile % g.strips, tile / g.strips, lane);
  }
}

template <typename T, int kWin, int TS, int CPL>
StepArgs<T> make_args(const StepLaunch& L) {
  constexpr int halo = 4 * TS;
  constexpr int strip_cols = kWave * CPL - 2 * halo;
  StepArgs<T> g;
  g.q2i = static_cast<const T*>(L.in[0]);
  g.q3i = static_cast<const T*>(L.in[1]);
  g.q4i = static_cast<const T*>(L.in[2]);
  g.n = static_cast<const T*>(L.n);
  g.q2o = static_cast<T*>(L.out[0]);
  g.q3o = static_cast<T*>(L.out[1]);
  g.q4o = static_cast<T*>(L.out[2]);
  // the descriptor range of a plane (with per-row descriptors only a row's is used)
  const size_t plane = static_cast<size_t>(L.pitch) * L.ny * sizeof(T);
  g.plane_bytes = static_cast<unsigned>(plane <= kMaxPlaneDescriptorBytes ? plane : 0);
  g.nx = L.nx;
  g.ny = L.ny;
  g.pitch = L.pitch;
  g.strips = (L.nx + strip_cols - 1) / strip_cols;
  // the requested rows plus both halos, rounded up to the unroll depth; the
  // segment then takes every row those iterations produce
  g.iters = ((L.rows_per_seg + 2 * halo + kWin - 1) / kWin) * kWin;
  g.rows_per_seg = g.iters - 2 * halo;
  g.segs = (L.ny + g.rows_per_seg - 1) / g.rows_per_seg;
  g.d4 = static_cast<T>(L.delta * 0.25);
  g.dc = L.triple ? -g.d4 : g.d4;
  return g;
}

template <typename T, int VMODE, int CLS, int kWin, int PF, int TS, int CPL>
hipError_t launch_typed(const StepLaunch& L, hipStream_t stream) {
  const StepArgs<T> g = make_args<T, kWin, TS, CPL>(L);
  const int blocks_per_seg = (g.strips + kWavesPerBlock - 1) / kWavesPerBlock;
  const int blocks = blocks_per_seg * g.segs;
  // planes beyond one descriptor's 2^31-byte range are addressed row by row
  const bool rows = static_cast<size_t>(L.pitch) * L.ny * sizeof(T) > kMaxPlaneDescriptorBytes;
  if (rows) {
    hipLaunchKernelGGL((qla_step_ez_kernel<T, VMODE, CLS, kWin, PF, TS, CPL, kRowDescriptors>),
                       dim3(blocks), dim3(kWave * kWavesPerBlock), 0, stream, g);
  } else {
    hipLaunchKernelGGL((qla_step_ez_kernel<T, VMODE, CLS, kWin, PF, TS, CPL, kPlaneDescriptors>),
                       dim3(blocks), dim3(kWave * kWavesPerBlock), 0, stream, g);
  }
  return hipGetLastError();
}

// Calls f.template operator()<T, VMODE, CLS, kWin, PF, TS, CPL>() for the compiled
// variant that matches the runtime choices. Window depth: the smallest that keeps
// every live row (PF + 4 TS + 2 rows).
template <typename T, int VMODE, int CLS, int CPL, typename F>
auto with_depth(int prefetch, int fused, F&& f) {
  if (fused == 2) {
    return prefetch == 2 ? f.template operator()<T, VMODE, CLS, 12, 2, 2, CPL>()
                         : f.template operator()<T, VMODE, CLS, 13, 3, 2, CPL>();
  }
  return prefetch == 2 ? f.template operator()<T, VMODE, CLS, 8, 2, 1, CPL>()
                       : f.template operator()<T, VMODE, CLS, 9, 3, 1, CPL>();
}

// Two columns per lane exist for FP32 single-lattice launches (kPairs) only.
template <typename T, bool kPairs, int VMODE, int CLS, typename F>
auto with_shape(int prefetch, int fused, int cols, F&& f) {
  if constexpr (kPairs && std::is_same_v<T, float>) {
    if (cols == 2) return with_depth<T, VMODE, CLS, 2>(prefetch, fused, f);
  }
  return with_depth<T, VMODE, CLS, 1>(prefetch, fused, f);
}

template <typename T, bool kPairs, typename F>
auto with_variant(int vmode, int angle_class, int prefetch, int fused, int cols, F&& f) {
  const bool large = angle_class == kLarge;
  switch (vmode) {
    case kVSkewHalf:
      return large ? with_shape<T, kPairs, kVSkewHalf, kLarge>(prefetch, fused, cols, f)
                   : with_shape<T, kPairs, kVSkewHalf, kSmall>(prefetch, fused, cols, f);
    case kVPaper:
      return large ? with_shape<T, kPairs, kVPaper, kLarge>(prefetch, fused, cols, f)
                   : with_shape<T, kPairs, kVPaper, kSmall>(prefetch, fused, cols, f);
    case kVBStream:
      return large ? with_shape<T, kPairs, kVBStream, kLarge>(prefetch, fused, cols, f)
                   : with_shape<T, kPairs, kVBStream, kSmall>(prefetch, fused, cols, f);
    default:
      return large ? with_shape<T, kPairs, kVNone, kLarge>(prefetch, fused, cols, f)
                   : with_shape<T, kPairs, kVNone, kSmall>(prefetch, fused, cols, f);
  }
}

template <typename T>
hipError_t launch_prec(const StepLaunch& L, hipStream_t stream) {
  return with_variant<T, true>(
      L.vmode, L.angle_class, L.prefetch, L.fused_steps, L.cols_per_lane,
      [&]<typename U, int VM, int CL, int W, int PF, int TS, int CPL>() {
        return launch_typed<U, VM, CL, W, PF, TS, CPL>(L, stream);
      });
}

template <typename T>
hipError_t launch_batch_prec(const BatchLaunch& B, hipStream_t stream) {
  return with_variant<T, false>(
      B.vmode, B.angle_class, B.prefetch, B.fused, 1,
      [&]<typename U, int VM, int CL, int W, int PF, int TS, int CPL>() -> hipError_t {
        auto kern = qla_batch_kernel<U, VM, CL, W, PF, TS>;
        const StepArgs<U>* args = static_cast<const StepArgs<U>*>(B.args);
        const unsigned* items = B.items;
        const int* counts = B.counts;
        const int* parity = B.parity;
        hipLaunchKernelGGL(kern, dim3(B.blocks), dim3(kWave * kWavesPerBlock), 0, stream, args,
                           items, counts, parity, B.pass);
        return hipGetLastError();
      });
}

template <typename T>
hipError_t batch_blocks_prec(const BatchLaunch& B, int* blocks) {
  return with_variant<T, false>(
      B.vmode, B.angle_class, B.prefetch, B.fused, 1,
      [&]<typename U, int VM, int CL, int W, int PF, int TS, int CPL>() -> hipError_t {
        int per_cu = 0, cus = 0, dev = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, qla_batch_kernel<U, VM, CL, W, PF, TS>, kWave * kWavesPerBlock, 0);
        if (e != hipSuccess) return e;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        *blocks = per_cu * cus;
        return hipSuccess;
      });
}

// Batch tables: one column per lane (instances of odd width share the kernel).
template <typename T>
void fill_args_prec(const StepLaunch& L, void* dst, int* tiles) {
  with_variant<T, false>(L.vmode, L.angle_class, L.prefetch, L.fused_steps, 1,
                         [&]<typename U, int VM, int CL, int W, int PF, int TS, int CPL>() {
                           const StepArgs<U> g = make_args<U, W, TS, 1>(L);
                           std::memcpy(dst, &g, sizeof(g));
                           *tiles = g.strips * g.segs;
                           return 0;
                         });
}

}  // namespace

hipError_t launch_step(const StepLaunch& L, hipStream_t stream) {
  return L.fp32 ? launch_prec<float>(L, stream) : launch_prec<double>(L, stream);
}

hipError_t launch_batch(const BatchLaunch& B, hipStream_t stream) {
  return B.fp32 ? launch_batch_prec<float>(B, stream) : launch_batch_prec<double>(B, stream);
}

hipError_t batch_resident_blocks(const BatchLaunch& B, int* blocks) {
  return B.fp32 ? batch_blocks_prec<float>(B, blocks) : batch_blocks_prec<double>(B, blocks);
}

size_t step_args_bytes(bool fp32) {
  return fp32 ? sizeof(StepArgs<float>) : sizeof(StepArgs<double>);
}

void fill_step_args(const StepLaunch& L, void* dst, int* tiles) {
  if (L.fp32) {
    fill_args_prec<float>(L, dst, tiles);
  } else {
    fill_args_prec<double>(L, dst, tiles);
  }
}

}  // namespace qla
