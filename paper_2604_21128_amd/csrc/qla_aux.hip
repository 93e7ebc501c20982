// Set-up, diagnostic and readout kernels around the fused step: index preparation
// and checks, the per-site coefficients of Eqs. (2e4) and (2e13), the initial
// packet, the energy of Eq. (A13) and field readout.
//
// Site (x, y) is element y * pitch + x of a lattice plane (rows padded to the pitch)
// and element y * nx + x of a packed array (host order: staging, readout, inputs).
// Every kernel deals rows to blocks and the columns of a row to the threads of a
// block, so accesses along a row are coalesced and no division is needed.
#include <hip/hip_runtime.h>

#include <cmath>

#include "qla_device.h"
#include "qla_internal.h"

namespace qla {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ unsigned long long bits(double v) {
  return __builtin_bit_cast(unsigned long long, v);
}

// Reduce within the block; for non-negative doubles, the order of the bit patterns
// as unsigned integers is the order of the values.
template <typename Op>
__device__ unsigned long long block_reduce_u64(unsigned long long v, Op op,
                                               unsigned long long* lds) {
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = op(v, o);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < static_cast<int>(blockDim.x >> 6); ++i) v = op(v, lds[i]);
  }
  return v;
}

struct MinOp {
  __device__ unsigned long long operator()(unsigned long long a, unsigned long long b) const {
    return a < b ? a : b;
  }
};
struct MaxOp {
  __device__ unsigned long long operator()(unsigned long long a, unsigned long long b) const {
    return a > b ? a : b;
  }
};
struct AddOp {
  __device__ unsigned long long operator()(unsigned long long a, unsigned long long b) const {
    return a + b;
  }
};

__global__ __launch_bounds__(kBlock) void index_copy_kernel(const double* __restrict__ src,
                                                            size_t ld, int nx, int ny,
                                                            size_t pitch,
                                                            double* __restrict__ n64,
                                                            float* __restrict__ n32,
                                                            unsigned long long* stats) {
  __shared__ unsigned long long lds[kBlock / 64];
  unsigned long long bad = 0, nmin = bits(INFINITY);
  for (int y = blockIdx.x; y < ny; y += gridDim.x) {
    for (int x = threadIdx.x; x < nx; x += kBlock) {
      const double v = src[static_cast<size_t>(y) * ld + x];
      const size_t i = static_cast<size_t>(y) * pitch + x;
      n64[i] = v;
      if (n32) n32[i] = static_cast<float>(v);
      if (!(v > 0.0) || !isfinite(v)) {
        ++bad;
      } else if (bits(v) < nmin) {
        nmin = bits(v);
      }
    }
  }
  bad = block_reduce_u64(bad, AddOp{}, lds);
  __syncthreads();
  nmin = block_reduce_u64(nmin, MinOp{}, lds);
  if (threadIdx.x == 0) {
    if (bad) atomicAdd(&stats[0], bad);
    atomicMin(&stats[1], nmin);
  }
}

// beta/2 along x and y exactly as the step computes it.
__device__ __forceinline__ void half_betas(const double* __restrict__ n, int nx, int ny,
                                           size_t pitch, int x, int y, double d4, double& hbx,
                                           double& hby, double& m) {
  const size_t row = static_cast<size_t>(y) * pitch;
  const int xl = x == 0 ? nx - 1 : x - 1, xr = x + 1 == nx ? 0 : x + 1;
  const int yl = y == 0 ? ny - 1 : y - 1, yr = y + 1 == ny ? 0 : y + 1;
  m = recip(n[row + x]);
  const double dm = d4 * m * m;
  hbx = (n[row + xr] - n[row + xl]) * dm;
  hby = (n[static_cast<size_t>(yr) * pitch + x] - n[static_cast<size_t>(yl) * pitch + x]) * dm;
}

__global__ __launch_bounds__(kBlock) void index_beta_max_kernel(const double* __restrict__ n64,
                                                                int nx, int ny, size_t pitch,
                                                                double d4,
                                                                unsigned long long* stats) {
  __shared__ unsigned long long lds[kBlock / 64];
  unsigned long long mx = 0;
  for (int y = blockIdx.x; y < ny; y += gridDim.x) {
    for (int x = threadIdx.x; x < nx; x += kBlock) {
      double hbx, hby, m;
      half_betas(n64, nx, ny, pitch, x, y, d4, hbx, hby, m);
      const double a = fmax(fabs(hbx), fabs(hby));
      const unsigned long long b = isfinite(a) ? bits(a) : bits(INFINITY);
      mx = b > mx ? b : mx;
    }
  }
  mx = block_reduce_u64(mx, MaxOp{}, lds);
  if (threadIdx.x == 0) atomicMax(&stats[2], mx);
}

__global__ __launch_bounds__(kBlock) void coefficients_kernel(const double* __restrict__ n64,
                                                              int nx, int ny, size_t pitch,
                                                              double d4, double* theta,
                                                              double* bx, double* by) {
  for (int y = blockIdx.x; y < ny; y += gridDim.x) {
    for (int x = threadIdx.x; x < nx; x += kBlock) {
      double hbx, hby, m;
      half_betas(n64, nx, ny, pitch, x, y, d4, hbx, hby, m);
      const size_t i = static_cast<size_t>(y) * nx + x;  // packed outputs
      if (theta) theta[i] = d4 * m;
      if (bx) bx[i] = hbx + hbx;
      if (by) by[i] = hby + hby;
    }
  }
}

// n(x, y) of an elliptical dielectric (or bubble) with a tanh boundary layer: the
// first-order signed distance d = (rho^2 - 1) / (2 |grad rho^2| / 2) to the ellipse
// rho^2 = (x'/a)^2 + (y'/b)^2 = 1 in coordinates rotated by rot about (xc, yc), and
// n = n_out + (n_in - n_out) (1 - tanh(d / width)) / 2 (n_in at the exact centre).
__global__ __launch_bounds__(kBlock) void ellipse_index_kernel(int nx, int ny, EllipseArgs e,
                                                               double* __restrict__ out) {
  const double cr = cos(e.rot), sr = sin(e.rot);
  for (int y = blockIdx.x; y < ny; y += gridDim.x)
  for (int x = threadIdx.x; x < nx; x += kBlock) {
    const size_t i = static_cast<size_t>(y) * nx + x;  // packed output
    const double dx = x - e.xc, dy = y - e.yc;
    const double xp = dx * cr + dy * sr, yp = -dx * sr + dy * cr;
    const double u = xp / e.a, v = yp / e.b;
    const double rho2 = u * u + v * v;
    const double gx = xp / (e.a * e.a), gy = yp / (e.b * e.b);
    const double g = sqrt(gx * gx + gy * gy);
    const double prof = g > 0.0 ? 0.5 * (1.0 - tanh((rho2 - 1.0) / (2.0 * g) / e.width)) : 1.0;
    out[i] = e.n_out + (e.n_in - e.n_out) * prof;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void packet_kernel(const double* __restrict__ n64, int nx,
                                                        int ny, size_t pitch, PacketArgs p, T* q2,
                                                        T* q3, T* q4) {
  const double kx = cos(p.phi), ky = sin(p.phi);
  const double two_pi = 6.283185307179586476925286766559;
  for (int y = blockIdx.x; y < ny; y += gridDim.x)
  for (int x = threadIdx.x; x < nx; x += kBlock) {
    const size_t i = static_cast<size_t>(y) * pitch + x;
    double dx = x - p.x0, dy = y - p.y0;
    dx -= nx * floor(dx / nx + 0.5);
    dy -= ny * floor(dy / ny + 0.5);
    const double s = dx * kx + dy * ky;
    const double r2 = p.planar ? s * s : dx * dx + dy * dy;
    const double f = p.amp * exp(-r2 / (2.0 * p.sigma * p.sigma)) * cos(two_pi * s / p.lambda);
    if (p.triple == 0) {
      // E_z packet: q2 = n Ez, (q3, q4) = q2 (sin phi, -cos phi)
      const double a = n64[i] * f;
      q2[i] = static_cast<T>(a);
      q3[i] = static_cast<T>(a * ky);
      q4[i] = static_cast<T>(-a * kx);
    } else {
      // B_z packet into (q5, q0, q1): q5 = Bz, (q0, q1) = n E = Bz (-sin phi, cos phi)
      q2[i] = static_cast<T>(f);
      q3[i] = static_cast<T>(-f * ky);
      q4[i] = static_cast<T>(f * kx);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void energy_partial_kernel(const T* __restrict__ q2,
                                                                const T* __restrict__ q3,
                                                                const T* __restrict__ q4,
                                                                int nx, int ny, size_t pitch,
                                                                double* partials) {
  __shared__ double lds[kBlock];
  double acc = 0.0;
  for (int y = blockIdx.x; y < ny; y += gridDim.x) {
    for (int x = threadIdx.x; x < nx; x += kBlock) {
      const size_t i = static_cast<size_t>(y) * pitch + x;
      const double a = q2[i], b = q3[i], c = q4[i];
      acc = fma(a, a, acc);
      acc = fma(b, b, acc);
      acc = fma(c, c, acc);
    }
  }
  lds[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = lds[0];
}

__global__ __launch_bounds__(kEnergyPartials) void energy_final_kernel(const double* partials,
                                                                       double* out) {
  __shared__ double lds[kEnergyPartials];
  lds[threadIdx.x] = partials[threadIdx.x];
  __syncthreads();
  for (int s = kEnergyPartials / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = lds[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void readout_kernel(const T* __restrict__ q2,
                                                         const T* __restrict__ q3,
                                                         const T* __restrict__ q4,
                                                         const double* __restrict__ n64,
                                                         int nx, int ny, size_t pitch,
                                                         int divide_by_n,
                                                         double* __restrict__ out) {
  const size_t count = static_cast<size_t>(nx) * ny;
  for (int y = blockIdx.x; y < ny; y += gridDim.x) {
    for (int x = threadIdx.x; x < nx; x += kBlock) {
      const size_t i = static_cast<size_t>(y) * pitch + x, o = static_cast<size_t>(y) * nx + x;
      const double a = q2[i], b = q3[i], c = q4[i];
      out[o] = (divide_by_n & 1) ? a / n64[i] : a;
      out[count + o] = (divide_by_n & 2) ? b / n64[i] : b;
      out[2 * count + o] = (divide_by_n & 4) ? c / n64[i] : c;
    }
  }
}

// Per-block partial sums of div^2 and of the squared axis derivatives, and partial
// maxima of |div|, for F = w (fx, fy): div = (Fx[x+1] - Fx[x-1] + Fy[y+1] - Fy[y-1]) / (2 delta)
// with Fx = w fx, Fy = w fy (periodic). One partial per block, fixed order.
template <typename T>
__global__ __launch_bounds__(kBlock) void divergence_partial_kernel(
    const T* __restrict__ fx, const T* __restrict__ fy, const double* __restrict__ n64, int nx,
    int ny, size_t pitch, double inv_2d, int weight_n, double* __restrict__ partials) {
  __shared__ double l0[kBlock], l1[kBlock], l2[kBlock];
  double s_div = 0.0, s_scale = 0.0, m_div = 0.0;
  for (int y = blockIdx.x; y < ny; y += gridDim.x)
  for (int x = threadIdx.x; x < nx; x += kBlock) {
    const size_t xl = static_cast<size_t>(y) * pitch + (x == 0 ? nx - 1 : x - 1);
    const size_t xr = static_cast<size_t>(y) * pitch + (x == nx - 1 ? 0 : x + 1);
    const size_t yd = static_cast<size_t>(y == 0 ? ny - 1 : y - 1) * pitch + x;
    const size_t yu = static_cast<size_t>(y == ny - 1 ? 0 : y + 1) * pitch + x;
    double fxr = fx[xr], fxl = fx[xl], fyu = fy[yu], fyd = fy[yd];
    if (weight_n) {
      fxr *= n64[xr];
      fxl *= n64[xl];
      fyu *= n64[yu];
      fyd *= n64[yd];
    }
    const double dfx = (fxr - fxl) * inv_2d, dfy = (fyu - fyd) * inv_2d;
    const double div = dfx + dfy;
    s_div = fma(div, div, s_div);
    s_scale = fma(dfx, dfx, fma(dfy, dfy, s_scale));
    m_div = fmax(m_div, fabs(div));
  }
  l0[threadIdx.x] = s_div;
  l1[threadIdx.x] = m_div;
  l2[threadIdx.x] = s_scale;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) {
      l0[threadIdx.x] += l0[threadIdx.x + s];
      l1[threadIdx.x] = fmax(l1[threadIdx.x], l1[threadIdx.x + s]);
      l2[threadIdx.x] += l2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = l0[0];
    partials[kEnergyPartials + blockIdx.x] = l1[0];
    partials[2 * kEnergyPartials + blockIdx.x] = l2[0];
  }
}

__global__ __launch_bounds__(kEnergyPartials) void divergence_final_kernel(
    const double* partials, double* out) {
  __shared__ double l0[kEnergyPartials], l1[kEnergyPartials], l2[kEnergyPartials];
  l0[threadIdx.x] = partials[threadIdx.x];
  l1[threadIdx.x] = partials[kEnergyPartials + threadIdx.x];
  l2[threadIdx.x] = partials[2 * kEnergyPartials + threadIdx.x];
  __syncthreads();
  for (int s = kEnergyPartials / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) {
      l0[threadIdx.x] += l0[threadIdx.x + s];
      l1[threadIdx.x] = fmax(l1[threadIdx.x], l1[threadIdx.x + s]);
      l2[threadIdx.x] += l2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = l0[0];
    out[1] = l1[0];
    out[2] = l2[0];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void from_f64_kernel(const double* __restrict__ src, int nx,
                                                          int ny, size_t pitch, T* q2, T* q3,
                                                          T* q4) {
  const size_t count = static_cast<size_t>(nx) * ny;
  for (int y = blockIdx.x; y < ny; y += gridDim.x) {
    for (int x = threadIdx.x; x < nx; x += kBlock) {
      const size_t i = static_cast<size_t>(y) * pitch + x, o = static_cast<size_t>(y) * nx + x;
      q2[i] = static_cast<T>(src[o]);
      q3[i] = static_cast<T>(src[count + o]);
      q4[i] = static_cast<T>(src[2 * count + o]);
    }
  }
}

// One block per row (up to 8192 blocks, which then stride over the rows).
unsigned grid_for(int ny) { return static_cast<unsigned>(ny < 8192 ? (ny > 0 ? ny : 1) : 8192); }

}  // namespace

hipError_t launch_index_prepare(const double* src, size_t ld, int nx, int ny, size_t pitch,
                                double delta, double* n64, float* n32,
                                unsigned long long* stats, hipStream_t stream) {
  hipLaunchKernelGGL(index_copy_kernel, dim3(grid_for(ny)), dim3(kBlock), 0, stream, src, ld,
                     nx, ny, pitch, n64, n32, stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(index_beta_max_kernel, dim3(grid_for(ny)), dim3(kBlock), 0, stream, n64,
                     nx, ny, pitch, 0.25 * delta, stats);
  return hipGetLastError();
}

hipError_t launch_coefficients(const double* n64, int nx, int ny, size_t pitch, double delta,
                               double* theta, double* beta_x, double* beta_y,
                               hipStream_t stream) {
  hipLaunchKernelGGL(coefficients_kernel, dim3(grid_for(ny)), dim3(kBlock), 0, stream, n64, nx,
                     ny, pitch, 0.25 * delta, theta, beta_x, beta_y);
  return hipGetLastError();
}

hipError_t launch_ellipse_index(int nx, int ny, const EllipseArgs& e, double* out,
                                hipStream_t stream) {
  hipLaunchKernelGGL(ellipse_index_kernel, dim3(grid_for(ny)), dim3(kBlock), 0, stream, nx, ny,
                     e, out);
  return hipGetLastError();
}

hipError_t launch_packet(const double* n64, int nx, int ny, size_t pitch, const PacketArgs& p,
                         bool fp32, void* q2, void* q3, void* q4, hipStream_t stream) {
  if (fp32) {
    hipLaunchKernelGGL(packet_kernel<float>, dim3(grid_for(ny)), dim3(kBlock), 0, stream, n64,
                       nx, ny, pitch, p, static_cast<float*>(q2), static_cast<float*>(q3),
                       static_cast<float*>(q4));
  } else {
    hipLaunchKernelGGL(packet_kernel<double>, dim3(grid_for(ny)), dim3(kBlock), 0, stream, n64,
                       nx, ny, pitch, p, static_cast<double*>(q2), static_cast<double*>(q3),
                       static_cast<double*>(q4));
  }
  return hipGetLastError();
}

hipError_t launch_energy(const void* q2, const void* q3, const void* q4, int nx, int ny,
                         size_t pitch, bool fp32, double* partials, double* out,
                         hipStream_t stream) {
  if (fp32) {
    hipLaunchKernelGGL(energy_partial_kernel<float>, dim3(kEnergyPartials), dim3(kBlock), 0,
                       stream, static_cast<const float*>(q2), static_cast<const float*>(q3),
                       static_cast<const float*>(q4), nx, ny, pitch, partials);
  } else {
    hipLaunchKernelGGL(energy_partial_kernel<double>, dim3(kEnergyPartials), dim3(kBlock), 0,
                       stream, static_cast<const double*>(q2), static_cast<const double*>(q3),
                       static_cast<const double*>(q4), nx, ny, pitch, partials);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kEnergyPartials), 0, stream, partials,
                     out);
  return hipGetLastError();
}

hipError_t launch_readout(const void* q2, const void* q3, const void* q4, const double* n64,
                          int nx, int ny, size_t pitch, bool fp32, int divide_by_n, double* out,
                          hipStream_t stream) {
  if (fp32) {
    hipLaunchKernelGGL(readout_kernel<float>, dim3(grid_for(ny)), dim3(kBlock), 0, stream,
                       static_cast<const float*>(q2), static_cast<const float*>(q3),
                       static_cast<const float*>(q4), n64, nx, ny, pitch, divide_by_n, out);
  } else {
    hipLaunchKernelGGL(readout_kernel<double>, dim3(grid_for(ny)), dim3(kBlock), 0, stream,
                       static_cast<const double*>(q2), static_cast<const double*>(q3),
                       static_cast<const double*>(q4), n64, nx, ny, pitch, divide_by_n, out);
  }
  return hipGetLastError();
}

hipError_t launch_divergence(const void* fx, const void* fy, const double* n64, int nx, int ny,
                             size_t pitch, double delta, bool fp32, bool weight_n,
                             double* partials, double* out, hipStream_t stream) {
  const double inv_2d = 0.5 / delta;
  if (fp32) {
    hipLaunchKernelGGL(divergence_partial_kernel<float>, dim3(kEnergyPartials), dim3(kBlock), 0,
                       stream, static_cast<const float*>(fx), static_cast<const float*>(fy), n64,
                       nx, ny, pitch, inv_2d, weight_n ? 1 : 0, partials);
  } else {
    hipLaunchKernelGGL(divergence_partial_kernel<double>, dim3(kEnergyPartials), dim3(kBlock), 0,
                       stream, static_cast<const double*>(fx), static_cast<const double*>(fy),
                       n64, nx, ny, pitch, inv_2d, weight_n ? 1 : 0, partials);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(divergence_final_kernel, dim3(1), dim3(kEnergyPartials), 0, stream, partials,
                     out);
  return hipGetLastError();
}

hipError_t launch_from_f64(const double* src, int nx, int ny, size_t pitch, bool fp32, void* q2,
                           void* q3, void* q4, hipStream_t stream) {
  if (fp32) {
    hipLaunchKernelGGL(from_f64_kernel<float>, dim3(grid_for(ny)), dim3(kBlock), 0, stream, src,
                       nx, ny, pitch, static_cast<float*>(q2), static_cast<float*>(q3),
                       static_cast<float*>(q4));
  } else {
    hipLaunchKernelGGL(from_f64_kernel<double>, dim3(grid_for(ny)), dim3(kBlock), 0, stream, src,
                       nx, ny, pitch, static_cast<double*>(q2), static_cast<double*>(q3),
                       static_cast<double*>(q4));
  }
  return hipGetLastError();
}

}  // namespace qla
