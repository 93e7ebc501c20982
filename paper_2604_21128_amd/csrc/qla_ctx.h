// The state of one lattice (shared by the single-lattice and batched C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "qla.h"
#include "qla_internal.h"

namespace qla {
constexpr int kDefaultRows = 24;
constexpr int kDefaultPrefetch = 3;
constexpr int kDefaultFused = 2;
}  // namespace qla

struct qla_ctx {
  int nx = 0, ny = 0;
  double delta = 0.0;
  bool fp32 = false;
  int vmode = 0;
  // 0: the E_z triple, planes (q2, q3, q4); 1: the B_z triple, stored as (q5, q0, q1) so
  // the step treats both alike (shared component first, then its y and x partners)
  int triple = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool owned_by_batch = false;
  void* q[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  int cur = 0;
  double* n64 = nullptr;
  float* n32 = nullptr;
  double* staging = nullptr;  // 3 * pitch * ny doubles: packed host-order arrays, scratch
  double* partials = nullptr;  // 3 * kEnergyPartials doubles (energy, divergence)
  double* diag = nullptr;      // 3 doubles: divergence results
  double* energy_dev = nullptr;
  unsigned long long* stats = nullptr;
  int64_t steps = 0;
  bool have_index = false;
  int angle_class = 0;
  int rows_per_seg = qla::kDefaultRows;
  int prefetch = qla::kDefaultPrefetch;
  int fused = qla::kDefaultFused;
  int cols = 1;  // lattice columns per lane of the step kernel (2: FP32, even nx only)
  // Row pitch of every lattice plane (amplitudes, n64, n32), in elements: nx rounded up
  // to a whole number of 128-byte cache lines of the stepping precision, so every row
  // starts on a line (an unaligned pitch measured ~15% slower).
  int pitch = 0;
  size_t count() const { return static_cast<size_t>(nx) * static_cast<size_t>(ny); }
  size_t plane_elems() const { return static_cast<size_t>(pitch) * static_cast<size_t>(ny); }
  size_t elem() const { return fp32 ? sizeof(float) : sizeof(double); }
  // The stored plane holding component j of the ABI order ((q2, q3, q4) or (q0, q1, q5)).
  int plane(int j) const { return triple == 0 ? j : (j + 1) % 3; }
};

namespace qla {

extern thread_local std::string g_last_error;
qla_status fail(qla_status s, const std::string& msg);
qla_status hip_fail(hipError_t e, const char* what);

#define QLA_HIP(call)                                         \
  do {                                                        \
    const hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::qla::hip_fail(e_, #call);  \
  } while (0)

// Makes a device current for the duration of a call.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
  bool ok() const { return ok_; }

 private:
  int prev_ = 0;
  bool ok_ = false;
};

// Makes device `dev` current until the enclosing call returns; the call fails with
// QLA_EDEVICE when the device cannot be selected.
#define QLA_ON_DEVICE(dev)                                                           \
  ::qla::DeviceGuard guard_(dev);                                                    \
  if (!guard_.ok()) return ::qla::fail(QLA_EDEVICE, "cannot select the device")

// Enqueue k steps of one context with the given tuning (no argument checks).
qla_status enqueue_steps(qla_ctx* c, int64_t k, int rows, int prefetch, int fused, int cols);

// The step launch for one pass of context c: dir 0 reads the current buffer, dir 1
// the other one.
StepLaunch step_launch_for(const qla_ctx* c, int rows, int prefetch, int fused, int dir);

}  // namespace qla
