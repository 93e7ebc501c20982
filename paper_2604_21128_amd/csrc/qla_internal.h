// Internal interface between the C ABI (qla_api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qla {

enum VMode : int { kVSkewHalf = 0, kVPaper = 1, kVNone = 2, kVBStream = 3 };

// One fused step (qla_step.hip): three amplitude planes in, three out, n in the
// stepping precision; all planes ny rows of `pitch` elements (nx of them used).
struct StepLaunch {
  const void* in[3];
  void* out[3];
  const void* n;
  int nx, ny;
  int pitch;         // row pitch of every plane, elements (>= nx)
  int rows_per_seg;  // requested output rows per wavefront segment (rounded up)
  int prefetch;      // rows the loads run ahead: 2 or 3
  int fused_steps;   // steps applied per pass: 1 or 2
  int cols_per_lane;  // lattice columns per lane: 1, or 2 (FP32, even nx)
  double delta;
  bool fp32;
  int vmode;
  int angle_class;
  int triple;  // 0: E_z triple (q2, q3, q4); 1: B_z triple (q5, q0, q1), collision angles negated
};
hipError_t launch_step(const StepLaunch& L, hipStream_t stream);

// Batched passes over many lattices (qla_step.hip, qla_batch_kernel). `args`
// points to 2 StepArgs per instance (filled by fill_step_args), `items` to the
// (instance << 20 | tile) list and `counts` to the number of items of each pass.
struct BatchLaunch {
  const void* args;
  const unsigned* items;
  const int* counts;
  const int* parity;  // per instance: 1 if its buffers are swapped relative to args
  int pass;      // the pass this launch runs
  int blocks;    // grid size (batch_resident_blocks: every wave stays resident)
  bool fp32;
  int vmode, angle_class, prefetch, fused;
};
hipError_t launch_batch(const BatchLaunch& B, hipStream_t stream);
hipError_t batch_resident_blocks(const BatchLaunch& B, int* blocks);
size_t step_args_bytes(bool fp32);
// The kernel's argument block for one pass of one lattice (in, out, n, sizes and the
// tuning in L) written to host memory at dst; *tiles = wavefront tiles per pass.
void fill_step_args(const StepLaunch& L, void* dst, int* tiles);

// Plane geometry of the auxiliary kernels (qla_aux.hip): lattice planes hold ny rows
// of `pitch` elements (nx used); packed arrays (staging, readout, inputs) hold ny
// rows of nx.
//
// Index preparation: copy n (row pitch ld) into the FP64 plane n64 (and its FP32
// rounding n32 when non-null), and accumulate into
// stats[0] the number of entries that are not finite or not > 0, into stats[1]
// the bit pattern of the smallest n and into stats[2] the bit pattern of the
// largest |beta/2| over both axes. stats must be preset to {0, +inf, 0}.
hipError_t launch_index_prepare(const double* src, size_t ld, int nx, int ny, size_t pitch,
                                double delta, double* n64, float* n32,
                                unsigned long long* stats, hipStream_t stream);

// theta = delta / (4 n), beta_x, beta_y = delta^2 (dn/dx, dn/dy) / n^2 (FP64), packed.
hipError_t launch_coefficients(const double* n64, int nx, int ny, size_t pitch, double delta,
                               double* theta, double* beta_x, double* beta_y,
                               hipStream_t stream);

struct EllipseArgs {
  double xc, yc, a, b, rot, n_in, n_out, width;
};
// n of an elliptical dielectric with a tanh boundary layer into a packed FP64 plane.
hipError_t launch_ellipse_index(int nx, int ny, const EllipseArgs& e, double* out,
                                hipStream_t stream);

struct PacketArgs {
  double x0, y0, sigma, lambda, phi, amp;
  int planar;
  int triple;  // 0: E_z packet into (q2, q3, q4); 1: B_z packet into (q5, q0, q1)
};
hipError_t launch_packet(const double* n64, int nx, int ny, size_t pitch, const PacketArgs& p,
                         bool fp32, void* q2, void* q3, void* q4, hipStream_t stream);

// Sum of squares of three planes over the lattice's sites, FP64, fixed order.
constexpr int kEnergyPartials = 1024;
hipError_t launch_energy(const void* q2, const void* q3, const void* q4, int nx, int ny,
                         size_t pitch, bool fp32, double* partials, double* out,
                         hipStream_t stream);

// Three planes to three packed FP64 arrays, in the order given; plane j is divided by
// n where bit j of divide_by_n is set (physical readout).
hipError_t launch_readout(const void* q2, const void* q3, const void* q4, const double* n64,
                          int nx, int ny, size_t pitch, bool fp32, int divide_by_n, double* out,
                          hipStream_t stream);

// Discrete divergence of the in-plane field F = w (fx, fy) with w = 1 (E_z triple:
// B = (q3, q4)) or w = n (B_z triple: D = n (q0, q1)), centred differences, periodic:
// out[0] = sum of div^2, out[1] = max |div|, out[2] = sum of (dFx/dx)^2 + (dFy/dy)^2,
// all FP64 in a fixed order. partials: 3 * kEnergyPartials doubles.
hipError_t launch_divergence(const void* fx, const void* fy, const double* n64, int nx, int ny,
                             size_t pitch, double delta, bool fp32, bool weight_n,
                             double* partials, double* out, hipStream_t stream);

// Packed FP64 staging (3 consecutive arrays) to the three amplitude planes.
hipError_t launch_from_f64(const double* src, int nx, int ny, size_t pitch, bool fp32, void* q2,
                           void* q3, void* q4, hipStream_t stream);

}  // namespace qla
