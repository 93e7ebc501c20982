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
//
// Mapping to the machine. A wavefront owns a strip of 56 output columns and a
// segment of output rows. Its 64 lanes hold columns x0-4 .. x0+59 (4 halo columns
// each side, periodic wrap), one column per lane. The wave marches down the rows:
//   - each incoming row gets U_x across the lanes, with the neighbour values
//     taken by DPP lane shifts (no LDS, no barriers);
//   - U_y runs down the rows inside each lane as a software pipeline: when row r
//     arrives, set 1 finishes row r-1, set 2 row r-2, set 3 row r-3 and set 4 row
//     r-4, which then gets V_x, V_y and is stored.
// The rows of the window live in registers, indexed modulo 8 with the loop
// unrolled 8 times so every index is static; loads run 2 rows ahead. The segment
// starts 4 rows early and ends 4 rows late (vertical halo). Rotations use the
// three-shear form (qla_device.h); angles come from n on the fly, so HBM traffic
// is exactly three amplitude planes in and out plus n in.
#include <hip/hip_runtime.h>

#include <utility>

#include "qla_device.h"
#include "qla_internal.h"

namespace qla {

namespace {

constexpr int kWave = 64;
constexpr int kHalo = 4;
constexpr int kStripCols = kWave - 2 * kHalo;  // 56 output columns per wave
constexpr int kWavesPerBlock = 4;
// A buffer store whose offset is at least the buffer's size is discarded by the
// hardware; stores of halo lanes and of rows outside the segment use this offset
// instead of a branch, so the memory counters stay static for the compiler.
constexpr unsigned kDropOffset = 0x80000000u;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* p, unsigned bytes) {
  // raw buffer (stride 0), 32-bit dwords, range-checked against `bytes`
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes),
                                           0x00020000);
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
}

template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
  if constexpr (sizeof(T) == 8) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
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
  unsigned plane_bytes;  // nx * ny * sizeof(T), at most 2^31
  int nx, ny, strips, segs, rows_per_seg, iters;
  T d4;  // delta / 4
};

// kWin: register window depth in rows (the loop is unrolled kWin times so every
// window index is static); PF: how many rows ahead the loads run.
template <typename T, int VMODE, int CLS, int kWin, int PF>
struct Marcher {
  static_assert(PF + 6 <= kWin, "a prefetched row must not overwrite a live one");
  // Row window: amplitudes, index, 1/n and the collision shear of each row.
  T A[kWin], P4[kWin], P3[kWin], N[kWin], M[kWin], Tt[kWin], Ts[kWin];
  __amdgpu_buffer_rsrc_t r2i, r3i, r4i, rn, r2o, r3o, r4o;
  unsigned col_bytes;    // this lane's column (wrapped) in bytes
  unsigned store_bytes;  // col_bytes for lanes that own an output column, else kDropOffset
  unsigned row_bytes;    // nx * sizeof(T)
  int yin;               // row index of the next row to load (wrapped)

  // y is uniform across the wave: the row offset is a scalar register and every
  // lane adds its fixed column offset.
  __device__ __forceinline__ void load_row(int slot, int y) {
    const unsigned soff = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(y)) * row_bytes;
    A[slot] = buf_load<T>(r2i, col_bytes, soff);
    P3[slot] = buf_load<T>(r3i, col_bytes, soff);
    P4[slot] = buf_load<T>(r4i, col_bytes, soff);
    N[slot] = buf_load<T>(rn, col_bytes, soff);
  }

  // U_x on the just-arrived row (slot s): lanes exchange neighbour values by DPP.
  __device__ __forceinline__ void ux(int s) {
    T a = A[s], p = P4[s];
    const T t0 = Tt[s], s0 = Ts[s];
    const T tl = from_left(t0), sl = from_left(s0);
    const T tr = from_right(t0), sr = from_right(s0);
    // set 1: C^T on site; C(th_i) on (a_i, p_{i-1})
    rotate(a, p, -t0, -s0);
    {
      const T pm = from_left(p), ap = from_right(a);
      const T an = rotate_first(a, pm, t0, s0);
      p = rotate_second(ap, p, tr, sr);
      a = an;
    }
    // set 2: C^T on site; C(th_{i-1}) on (a_i, p_{i-1})
    rotate(a, p, -t0, -s0);
    {
      const T pm = from_left(p), ap = from_right(a);
      const T an = rotate_first(a, pm, tl, sl);
      p = rotate_second(ap, p, t0, s0);
      a = an;
    }
    // set 3: C on site; C^T(th_i) on (a_i, p_{i+1})
    rotate(a, p, t0, s0);
    {
      const T pp = from_right(p), am = from_left(a);
      const T an = rotate_first(a, pp, -t0, -s0);
      p = rotate_second(am, p, -tl, -sl);
      a = an;
    }
    // set 4: C on site; C^T(th_{i+1}) on (a_i, p_{i+1})
    rotate(a, p, t0, s0);
    {
      const T pp = from_right(p), am = from_left(a);
      const T an = rotate_first(a, pp, -tr, -sr);
      p = rotate_second(am, p, -t0, -s0);
      a = an;
    }
    A[s] = a;
    P4[s] = p;
  }

  // U_y pipeline after row r (slot s0) arrived; C_y = R(-th), C_y^T = R(+th).
  template <int S0>
  __device__ __forceinline__ void uy() {
    constexpr int s0 = S0, s1 = (S0 + kWin - 1) % kWin, s2 = (S0 + kWin - 2) % kWin;
    constexpr int s3 = (S0 + kWin - 3) % kWin, s4 = (S0 + kWin - 4) % kWin;
    // set 1 on row r: on-site C_y^T, then (a_r, p_{r-1}) with C_y(th_r)
    rotate(A[s0], P3[s0], Tt[s0], Ts[s0]);
    rotate(A[s0], P3[s1], -Tt[s0], -Ts[s0]);
    // set 2 on row r-1: on-site C_y^T, then (a_{r-1}, p_{r-2}) with C_y(th_{r-2})
    rotate(A[s1], P3[s1], Tt[s1], Ts[s1]);
    rotate(A[s1], P3[s2], -Tt[s2], -Ts[s2]);
    // set 3 on row r-2: on-site C_y, then (a_{r-3}, p_{r-2}) with C_y^T(th_{r-3})
    rotate(A[s2], P3[s2], -Tt[s2], -Ts[s2]);
    rotate(A[s3], P3[s2], Tt[s3], Ts[s3]);
    // set 4 on row r-3: on-site C_y, then (a_{r-4}, p_{r-3}) with C_y^T(th_{r-3})
    rotate(A[s3], P3[s3], -Tt[s3], -Ts[s3]);
    rotate(A[s4], P3[s3], Tt[s3], Ts[s3]);
  }

  // V_x, V_y on the completed row r-4.
  template <int S0>
  __device__ __forceinline__ void potentials(T d4) {
    if constexpr (VMODE == kVNone) {
      return;
    } else {
      constexpr int s3 = (S0 + kWin - 3) % kWin, s4 = (S0 + kWin - 4) % kWin;
      constexpr int s5 = (S0 + kWin - 5) % kWin;
      const T m = M[s4];
      const T dm = d4 * m * m;
      const T nl = from_left(N[s4]), nr = from_right(N[s4]);
      const T hbx = (nr - nl) * dm;          // beta_x / 2
      const T hby = (N[s3] - N[s5]) * dm;    // beta_y / 2
      if constexpr (VMODE == kVSkewHalf) {
        const Shear<T> vx = shear_of<T, CLS>(hbx);
        rotate(A[s4], P4[s4], -vx.t, -vx.s);
        const Shear<T> vy = shear_of<T, CLS>(hby);
        rotate(A[s4], P3[s4], vy.t, vy.s);
      } else {
        const T bx = hbx + hbx, by = hby + hby;
        const T sbx = sin_series<T, CLS>(bx), cbx = cos_series<T, CLS>(bx);
        P4[s4] = fma(-sbx, A[s4], cbx * P4[s4]);
        const T sby = sin_series<T, CLS>(by), cby = cos_series<T, CLS>(by);
        P3[s4] = fma(sby, A[s4], cby * P3[s4]);
      }
    }
  }

  template <int S0>
  __device__ __forceinline__ void iteration(const StepArgs<T>& g, int r, int y0, int yend) {
    constexpr int s0 = S0, s4 = (S0 + kWin - 4) % kWin, sp = (S0 + PF) % kWin;
    // loads for row r + PF (the slot held row r + PF - kWin, no longer needed).
    // Issued unconditionally, also past the segment's end (rows wrap, so they stay
    // in bounds): a branch here would make the compiler wait for them at once.
    load_row(sp, yin);
    yin = (yin + 1 == g.ny) ? 0 : yin + 1;
    // collision shear of row r
    const T m = recip(N[s0]);
    M[s0] = m;
    const Shear<T> c = shear_of<T, CLS>(g.d4 * m);
    Tt[s0] = c.t;
    Ts[s0] = c.s;
    ux(s0);
    uy<S0>();
    // row r - 4 is complete: output row y0 + r - 8
    potentials<S0>(g.d4);
    const int yo = y0 + r - 2 * kHalo;
    const bool row_ok = yo >= y0 && yo < yend;
    const unsigned soff = row_ok ? static_cast<unsigned>(yo) * row_bytes : 0u;
    const unsigned voff = row_ok ? store_bytes : kDropOffset;
    buf_store<T>(A[s4], r2o, voff, soff);
    buf_store<T>(P3[s4], r3o, voff, soff);
    buf_store<T>(P4[s4], r4o, voff, soff);
  }
};

template <typename T, int VMODE, int CLS, int kWin, int PF>
__global__ __launch_bounds__(kWave * kWavesPerBlock) void qla_step_ez_kernel(StepArgs<T> g) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = threadIdx.x / kWave;
  const int blk = xcd_contiguous_block(blockIdx.x, gridDim.x);
  const int blocks_per_seg = (g.strips + kWavesPerBlock - 1) / kWavesPerBlock;
  const int seg = blk / blocks_per_seg;
  const int strip = (blk % blocks_per_seg) * kWavesPerBlock + wib;
  if (seg >= g.segs || strip >= g.strips) return;  // whole wave exits together

  Marcher<T, VMODE, CLS, kWin, PF> w;
  const int x0 = strip * kStripCols;
  int col = (x0 - kHalo + lane) % g.nx;
  if (col < 0) col += g.nx;
  const bool store_lane =
      lane >= kHalo && lane < kHalo + kStripCols && x0 + lane - kHalo < g.nx;
  w.col_bytes = static_cast<unsigned>(col) * sizeof(T);
  w.store_bytes = store_lane ? w.col_bytes : kDropOffset;
  w.row_bytes = static_cast<unsigned>(g.nx) * sizeof(T);
  w.r2i = plane_rsrc(g.q2i, g.plane_bytes);
  w.r3i = plane_rsrc(g.q3i, g.plane_bytes);
  w.r4i = plane_rsrc(g.q4i, g.plane_bytes);
  w.rn = plane_rsrc(g.n, g.plane_bytes);
  w.r2o = plane_rsrc(g.q2o, g.plane_bytes);
  w.r3o = plane_rsrc(g.q3o, g.plane_bytes);
  w.r4o = plane_rsrc(g.q4o, g.plane_bytes);
  const int y0 = seg * g.rows_per_seg;
  const int yend = min(y0 + g.rows_per_seg, g.ny);
#pragma unroll
  for (int k = 0; k < kWin; ++k) {
    w.A[k] = w.P4[k] = w.P3[k] = w.N[k] = w.M[k] = w.Tt[k] = w.Ts[k] = T(0);
  }
  int y = y0 - kHalo;
  if (y < 0) y += g.ny;
  // The prologue issues the first PF rows in the same pattern as the loop body
  // (4 loads, then 3 stores, here discarded ones), so the compiler sees the same
  // outstanding memory operations on entry as on the back edge and keeps its
  // waits at the prefetch distance instead of draining the queue every trip.
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    w.load_row(k, y);
    y = (y + 1 == g.ny) ? 0 : y + 1;
    buf_store<T>(T(0), w.r2o, kDropOffset, 0u);
    buf_store<T>(T(0), w.r3o, kDropOffset, 0u);
    buf_store<T>(T(0), w.r4o, kDropOffset, 0u);
  }
  w.yin = y;

  for (int r = 0; r < g.iters; r += kWin) {
    [&]<int... K>(std::integer_sequence<int, K...>) {
      (w.template iteration<K>(g, r + K, y0, yend), ...);
    }(std::make_integer_sequence<int, kWin>{});
  }
}

template <typename T, int VMODE, int CLS, int kWin, int PF>
hipError_t launch_typed(const StepLaunch& L, hipStream_t stream) {
  StepArgs<T> g;
  g.q2i = static_cast<const T*>(L.in[0]);
  g.q3i = static_cast<const T*>(L.in[1]);
  g.q4i = static_cast<const T*>(L.in[2]);
  g.n = static_cast<const T*>(L.n);
  g.q2o = static_cast<T*>(L.out[0]);
  g.q3o = static_cast<T*>(L.out[1]);
  g.q4o = static_cast<T*>(L.out[2]);
  g.plane_bytes = static_cast<unsigned>(static_cast<size_t>(L.nx) * L.ny * sizeof(T));
  g.nx = L.nx;
  g.ny = L.ny;
  g.strips = (L.nx + kStripCols - 1) / kStripCols;
  // the requested rows plus both halos, rounded up to the unroll depth; the
  // segment then takes every row those iterations produce
  g.iters = ((L.rows_per_seg + 2 * kHalo + kWin - 1) / kWin) * kWin;
  g.rows_per_seg = g.iters - 2 * kHalo;
  g.segs = (L.ny + g.rows_per_seg - 1) / g.rows_per_seg;
  g.d4 = static_cast<T>(L.delta * 0.25);
  const int blocks_per_seg = (g.strips + kWavesPerBlock - 1) / kWavesPerBlock;
  const int blocks = blocks_per_seg * g.segs;
  hipLaunchKernelGGL((qla_step_ez_kernel<T, VMODE, CLS, kWin, PF>), dim3(blocks),
                     dim3(kWave * kWavesPerBlock), 0, stream, g);
  return hipGetLastError();
}

template <typename T, int kWin, int PF>
hipError_t launch_pf(const StepLaunch& L, hipStream_t stream) {
  const bool large = L.angle_class == kLarge;
  switch (L.vmode) {
    case kVSkewHalf:
      return large ? launch_typed<T, kVSkewHalf, kLarge, kWin, PF>(L, stream)
                   : launch_typed<T, kVSkewHalf, kSmall, kWin, PF>(L, stream);
    case kVPaper:
      return large ? launch_typed<T, kVPaper, kLarge, kWin, PF>(L, stream)
                   : launch_typed<T, kVPaper, kSmall, kWin, PF>(L, stream);
    default:
      return large ? launch_typed<T, kVNone, kLarge, kWin, PF>(L, stream)
                   : launch_typed<T, kVNone, kSmall, kWin, PF>(L, stream);
  }
}

template <typename T>
hipError_t launch_prec(const StepLaunch& L, hipStream_t stream) {
  switch (L.prefetch) {
    case 2: return launch_pf<T, 8, 2>(L, stream);
    case 3: return launch_pf<T, 12, 3>(L, stream);
    default: return launch_pf<T, 12, 4>(L, stream);
  }
}

}  // namespace

hipError_t launch_step(const StepLaunch& L, hipStream_t stream) {
  return L.fp32 ? launch_prec<float>(L, stream) : launch_prec<double>(L, stream);
}



}  // namespace qla
