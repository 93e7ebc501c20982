// The energy of Eq. (A13) of three caller-owned planes, with no allocation: the FP64
// partial sums live in a file-scope device array instead of a context's buffer.
//
// For callers that cannot allocate device memory (code under HIP graph capture, tight
// serving loops). The array is this library's copy on each GPU; host code never
// passes its name to a kernel (on the host the name is only a stand-in): the device
// address is looked up once per device with hipGetSymbolAddress and cached.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "qla.h"
#include "qla_ctx.h"
#include "qla_internal.h"

namespace {

// The partial sums of one energy evaluation: one FP64 value per block of the partial
// kernel. Every call overwrites all of them before they are read, so nothing needs
// clearing between calls; calls that overlap on one GPU share the array and race.
__device__ __align__(256) double scratch[qla::kEnergyPartials];
// The partial kernel runs a fixed grid of kEnergyPartials blocks whatever the lattice
// size, so the array always holds what a call needs.
static_assert(sizeof(scratch) == qla::kEnergyPartials * sizeof(double), "one slot per block");

constexpr int kMaxDevices = 64;
std::mutex g_lock;
double* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev` (looked up on the first
// call on that device, with it current).
qla_status scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return qla::fail(QLA_EDEVICE, "device index " + std::to_string(dev) + " beyond " +
                                      std::to_string(kMaxDevices));
  std::lock_guard<std::mutex> hold(g_lock);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return qla::hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return QLA_OK;
}

}  // namespace

extern "C" {

qla_status qla_energy_noalloc(const void* q_a, const void* q_b, const void* q_c, int nx, int ny,
                              size_t pitch, qla_precision precision, double* energy_device,
                              void* hip_stream) {
  if (!q_a || !q_b || !q_c || !energy_device) return qla::fail(QLA_EINVAL, "NULL argument");
  if (nx < 1 || ny < 1) return qla::fail(QLA_EINVAL, "nx and ny must be >= 1");
  if (pitch < static_cast<size_t>(nx)) return qla::fail(QLA_EINVAL, "pitch < nx");
  if (precision != QLA_F64 && precision != QLA_F32)
    return qla::fail(QLA_EINVAL, "precision must be QLA_F64 or QLA_F32");
  int dev = 0;
  const hipError_t ge = hipGetDevice(&dev);
  if (ge != hipSuccess) return qla::hip_fail(ge, "hipGetDevice");
  double* partials = nullptr;
  const qla_status st = scratch_on(dev, &partials);
  if (st != QLA_OK) return st;
  const hipError_t e = qla::launch_energy(q_a, q_b, q_c, nx, ny, pitch, precision == QLA_F32,
                                          partials, energy_device,
                                          static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return qla::hip_fail(e, "energy launch");
  return QLA_OK;
}

}  // extern "C"
