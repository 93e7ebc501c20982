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

#include "qla_device.h"
#include "qla_internal.h"

namespace qla {

namespace {

constexpr int kWave = 64;
constexpr int kHalo = 4;
constexpr int kStripCols = kWave - 2 * kHalo;  // 56 output columns per wave
constexpr int kWavesPerBlock = 4;
constexpr int kWin = 8;  // register window depth (rows), power of two

template <typename T>
struct StepArgs {
  const T* __restrict__ q2i;
  const T* __restrict__ q3i;
  const T* __restrict__ q4i;
  const T* __restrict__ n;
  T* __restrict__ q2o;
  T* __restrict__ q3o;
  T* __restrict__ q4o;
  int nx, ny, strips, segs, rows_per_seg, iters;
  T d4;  // delta / 4
};

template <typename T, int VMODE, int CLS>
struct Marcher {
  // Row window: amplitudes, index, 1/n and the collision shear of each row.
  T A[kWin], P4[kWin], P3[kWin], N[kWin], M[kWin], Tt[kWin], Ts[kWin];
  int col;       // this lane's column (wrapped)
  int yin;       // row index of the next row to load (wrapped)
  bool store_lane;

  // y is uniform across the wave: the row offset stays in scalar registers and
  // every lane adds its fixed column.
  __device__ __forceinline__ void load_row(const StepArgs<T>& g, int slot, int y) {
    const size_t row = static_cast<size_t>(__builtin_amdgcn_readfirstlane(y)) * g.nx;
    A[slot] = (g.q2i + row)[col];
    P3[slot] = (g.q3i + row)[col];
    P4[slot] = (g.q4i + row)[col];
    N[slot] = (g.n + row)[col];
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
    constexpr int s0 = S0, s4 = (S0 + kWin - 4) % kWin, sp = (S0 + 2) % kWin;
    // loads for row r + 2 (the slot held row r - 6, no longer needed). Issued
    // unconditionally, also past the segment's end (rows wrap, so they stay in
    // bounds): a branch here would make the compiler wait for these loads at once.
    load_row(g, sp, yin);
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
    if (yo >= y0 && yo < yend && store_lane) {
      const size_t row = static_cast<size_t>(__builtin_amdgcn_readfirstlane(yo)) * g.nx;
      (g.q2o + row)[col] = A[s4];
      (g.q3o + row)[col] = P3[s4];
      (g.q4o + row)[col] = P4[s4];
    }
  }
};

template <typename T, int VMODE, int CLS>
__global__ __launch_bounds__(kWave * kWavesPerBlock) void qla_step_ez_kernel(StepArgs<T> g) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = threadIdx.x / kWave;
  const int blk = xcd_contiguous_block(blockIdx.x, gridDim.x);
  const int blocks_per_seg = (g.strips + kWavesPerBlock - 1) / kWavesPerBlock;
  const int seg = blk / blocks_per_seg;
  const int strip = (blk % blocks_per_seg) * kWavesPerBlock + wib;
  if (seg >= g.segs || strip >= g.strips) return;  // whole wave exits together

  Marcher<T, VMODE, CLS> w;
  const int x0 = strip * kStripCols;
  int col = (x0 - kHalo + lane) % g.nx;
  if (col < 0) col += g.nx;
  w.col = col;
  w.store_lane = lane >= kHalo && lane < kHalo + kStripCols && x0 + lane - kHalo < g.nx;
  const int y0 = seg * g.rows_per_seg;
  const int yend = min(y0 + g.rows_per_seg, g.ny);
#pragma unroll
  for (int k = 0; k < kWin; ++k) {
    w.A[k] = w.P4[k] = w.P3[k] = w.N[k] = w.M[k] = w.Tt[k] = w.Ts[k] = T(0);
  }
  int y = y0 - kHalo;
  if (y < 0) y += g.ny;
  w.load_row(g, 0, y);
  y = (y + 1 == g.ny) ? 0 : y + 1;
  w.load_row(g, 1, y);
  w.yin = (y + 1 == g.ny) ? 0 : y + 1;

  for (int r = 0; r < g.iters; r += kWin) {
    w.template iteration<0>(g, r + 0, y0, yend);
    w.template iteration<1>(g, r + 1, y0, yend);
    w.template iteration<2>(g, r + 2, y0, yend);
    w.template iteration<3>(g, r + 3, y0, yend);
    w.template iteration<4>(g, r + 4, y0, yend);
    w.template iteration<5>(g, r + 5, y0, yend);
    w.template iteration<6>(g, r + 6, y0, yend);
    w.template iteration<7>(g, r + 7, y0, yend);
  }
}

template <typename T, int VMODE, int CLS>
hipError_t launch_typed(const StepLaunch& L, hipStream_t stream) {
  StepArgs<T> g;
  g.q2i = static_cast<const T*>(L.in[0]);
  g.q3i = static_cast<const T*>(L.in[1]);
  g.q4i = static_cast<const T*>(L.in[2]);
  g.n = static_cast<const T*>(L.n);
  g.q2o = static_cast<T*>(L.out[0]);
  g.q3o = static_cast<T*>(L.out[1]);
  g.q4o = static_cast<T*>(L.out[2]);
  g.nx = L.nx;
  g.ny = L.ny;
  g.strips = (L.nx + kStripCols - 1) / kStripCols;
  g.rows_per_seg = L.rows_per_seg;
  g.segs = (L.ny + L.rows_per_seg - 1) / L.rows_per_seg;
  // rows_per_seg + 2 halos, rounded up to the unroll depth
  g.iters = ((L.rows_per_seg + 2 * kHalo + kWin - 1) / kWin) * kWin;
  g.d4 = static_cast<T>(L.delta * 0.25);
  const int blocks_per_seg = (g.strips + kWavesPerBlock - 1) / kWavesPerBlock;
  const int blocks = blocks_per_seg * g.segs;
  hipLaunchKernelGGL((qla_step_ez_kernel<T, VMODE, CLS>), dim3(blocks),
                     dim3(kWave * kWavesPerBlock), 0, stream, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prec(const StepLaunch& L, hipStream_t stream) {
  const bool large = L.angle_class == kLarge;
  switch (L.vmode) {
    case kVSkewHalf:
      return large ? launch_typed<T, kVSkewHalf, kLarge>(L, stream)
                   : launch_typed<T, kVSkewHalf, kSmall>(L, stream);
    case kVPaper:
      return large ? launch_typed<T, kVPaper, kLarge>(L, stream)
                   : launch_typed<T, kVPaper, kSmall>(L, stream);
    default:
      return large ? launch_typed<T, kVNone, kLarge>(L, stream)
                   : launch_typed<T, kVNone, kSmall>(L, stream);
  }
}

}  // namespace

hipError_t launch_step(const StepLaunch& L, hipStream_t stream) {
  return L.fp32 ? launch_prec<float>(L, stream) : launch_prec<double>(L, stream);
}

int step_rows_granularity() { return kWin; }

}  // namespace qla
