// C ABI of the QLA library (declared in include/qla.h): context lifetime, argument
// checks, device memory and the order of kernel launches on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "qla.h"
#include "qla_internal.h"

#include "qla_ctx.h"

namespace qla {

thread_local std::string g_last_error;

qla_status fail(qla_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

qla_status hip_fail(hipError_t e, const char* what) {
  return fail(QLA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

DeviceGuard::DeviceGuard(int dev) {
  ok_ = hipGetDevice(&prev_) == hipSuccess;
  if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
}

DeviceGuard::~DeviceGuard() {
  int now = prev_;
  if (hipGetDevice(&now) == hipSuccess && now != prev_) (void)hipSetDevice(prev_);
}

}  // namespace qla

using qla::DeviceGuard;
using qla::fail;
using qla::hip_fail;
using qla::g_last_error;

namespace {

void release(qla_ctx* c) {
  for (auto& buf : c->q)
    for (auto& p : buf)
      if (p) (void)hipFree(p);
  if (c->n64) (void)hipFree(c->n64);
  if (c->n32) (void)hipFree(c->n32);
  if (c->staging) (void)hipFree(c->staging);
  if (c->partials) (void)hipFree(c->partials);
  if (c->diag) (void)hipFree(c->diag);
  if (c->energy_dev) (void)hipFree(c->energy_dev);
  if (c->stats) (void)hipFree(c->stats);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

// Physical readout: E = q / n for the E components ((q2) or (q0, q1)); B as stored.
int divide_mask(const qla_ctx* c, int physical) {
  if (!physical) return 0;
  return c->triple == 0 ? 1 : 3;
}

qla_status alloc(void** p, size_t bytes, const char* what) {
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(QLA_ENOMEM, std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
  }
  return QLA_OK;
}

// Validates the index held in the scratch planes (raw input already copied there
// or readable at src) and installs it.
qla_status install_index(qla_ctx* c, const double* src, size_t ld) {
  // staging: the packed input in [0, N), the new planes after it (N <= P)
  const size_t P = c->plane_elems();
  double* n_new = c->staging + P;
  float* n32_new = c->fp32 ? reinterpret_cast<float*>(c->staging + 2 * P) : nullptr;
  const unsigned long long init[3] = {0ull, 0x7FF0000000000000ull, 0ull};  // 0, +inf, 0
  // Host data goes in with blocking copies once the stream is idle, so it has landed
  // before the kernels below read it whatever path the runtime takes for pageable memory.
  QLA_HIP(hipStreamSynchronize(c->stream));
  QLA_HIP(hipMemcpy(c->stats, init, sizeof(init), hipMemcpyHostToDevice));
  QLA_HIP(qla::launch_index_prepare(src, ld, c->nx, c->ny, c->pitch, c->delta, n_new, n32_new,
                                    c->stats, c->stream));
  unsigned long long got[3];
  QLA_HIP(hipMemcpyAsync(got, c->stats, sizeof(got), hipMemcpyDeviceToHost, c->stream));
  QLA_HIP(hipStreamSynchronize(c->stream));
  if (got[0] != 0)
    return fail(QLA_EINVAL, "refractive index: " + std::to_string(got[0]) +
                                " entries are not finite or not > 0");
  double nmin, hb;
  std::memcpy(&nmin, &got[1], sizeof(double));
  std::memcpy(&hb, &got[2], sizeof(double));
  const double theta = c->delta / (4.0 * nmin);
  int cls;
  if (theta <= 1.0 / 16.0 && hb <= 1.0 / 16.0) {
    cls = 0;
  } else if (theta <= 0.5 && hb <= 0.5) {
    cls = 1;
  } else {
    return fail(QLA_EINVAL, "lattice angles too large: max collision angle delta/(4n) = " +
                                std::to_string(theta) + ", max potential half-angle = " +
                                std::to_string(hb) + " (both must be <= 0.5 rad)");
  }
  QLA_HIP(hipMemcpyAsync(c->n64, n_new, P * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (c->fp32)
    QLA_HIP(hipMemcpyAsync(c->n32, n32_new, P * sizeof(float), hipMemcpyDeviceToDevice,
                           c->stream));
  QLA_HIP(hipStreamSynchronize(c->stream));
  c->angle_class = cls;
  c->have_index = true;
  c->steps = 0;
  return QLA_OK;
}

}  // namespace

namespace qla {

// Enqueue k steps on the context's stream with the given tuning (no checks).
qla_status enqueue_steps(qla_ctx* c, int64_t k, int rows, int prefetch, int fused, int cols) {
  qla::StepLaunch L{};
  L.n = c->fp32 ? static_cast<const void*>(c->n32) : static_cast<const void*>(c->n64);
  L.nx = c->nx;
  L.ny = c->ny;
  L.pitch = c->pitch;
  L.rows_per_seg = rows;
  L.prefetch = prefetch;
  L.cols_per_lane = cols;
  L.delta = c->delta;
  L.fp32 = c->fp32;
  L.vmode = c->vmode;
  L.angle_class = c->angle_class;
  L.triple = c->triple;
  // passes of `fused` steps, then single steps for the remainder
  int64_t done = 0;
  while (done < k) {
    L.fused_steps = (k - done >= fused) ? fused : 1;
    for (int j = 0; j < 3; ++j) {
      L.in[j] = c->q[c->cur][j];
      L.out[j] = c->q[c->cur ^ 1][j];
    }
    QLA_HIP(qla::launch_step(L, c->stream));
    c->cur ^= 1;
    c->steps += L.fused_steps;
    done += L.fused_steps;
  }
  return QLA_OK;
}

qla::StepLaunch step_launch_for(const qla_ctx* c, int rows, int prefetch, int fused, int dir) {
  qla::StepLaunch L{};
  L.n = c->fp32 ? static_cast<const void*>(c->n32) : static_cast<const void*>(c->n64);
  L.nx = c->nx;
  L.ny = c->ny;
  L.pitch = c->pitch;
  L.rows_per_seg = rows;
  L.prefetch = prefetch;
  L.fused_steps = fused;
  L.cols_per_lane = 1;
  L.delta = c->delta;
  L.fp32 = c->fp32;
  L.vmode = c->vmode;
  L.angle_class = c->angle_class;
  L.triple = c->triple;
  const int from = c->cur ^ dir;
  for (int j = 0; j < 3; ++j) {
    L.in[j] = c->q[from][j];
    L.out[j] = c->q[from ^ 1][j];
  }
  return L;
}

}  // namespace qla

using qla::enqueue_steps;

extern "C" {

const char* qla_strerror(qla_status s) {
  switch (s) {
    case QLA_OK: return "success";
    case QLA_EINVAL: return "invalid argument";
    case QLA_ENOMEM: return "out of memory";
    case QLA_EDEVICE: return "HIP device error";
    case QLA_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* qla_last_error(void) { return g_last_error.c_str(); }

qla_status qla_create(int nx, int ny, double delta, qla_precision precision,
                      qla_potential potential, void* hip_stream, qla_ctx** out) {
  return qla_create_triple(nx, ny, delta, precision, potential, QLA_TRIPLE_EZ, hip_stream, out);
}

qla_status qla_create_triple(int nx, int ny, double delta, qla_precision precision,
                             qla_potential potential, qla_triple triple, void* hip_stream,
                             qla_ctx** out) {
  if (!out) return fail(QLA_EINVAL, "out is NULL");
  *out = nullptr;
  if (nx < 8 || ny < 8) return fail(QLA_EINVAL, "nx and ny must be >= 8");
  if (static_cast<long long>(nx) * sizeof(double) >= (1ll << 31))
    return fail(QLA_EINVAL, "one row must stay below 2 GiB (nx < 2^28)");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(QLA_EINVAL, "delta must be > 0");
  if (precision != QLA_F64 && precision != QLA_F32) return fail(QLA_EINVAL, "bad precision");
  if (potential != QLA_V_SKEW_HALF && potential != QLA_V_PAPER && potential != QLA_V_NONE &&
      potential != QLA_V_BSTREAM)
    return fail(QLA_EINVAL, "bad potential mode");
  if (triple != QLA_TRIPLE_EZ && triple != QLA_TRIPLE_BZ) return fail(QLA_EINVAL, "bad triple");
  if (triple == QLA_TRIPLE_BZ && (potential == QLA_V_PAPER || potential == QLA_V_BSTREAM))
    return fail(QLA_EINVAL, "the printed potentials and the B-streaming scheme are implemented "
                            "for the E_z triple only");
  qla_ctx* c = new (std::nothrow) qla_ctx;
  if (!c) return fail(QLA_ENOMEM, "host allocation");
  c->nx = nx;
  c->ny = ny;
  c->delta = delta;
  c->fp32 = precision == QLA_F32;
  c->vmode = static_cast<int>(potential);
  c->triple = static_cast<int>(triple);
  {
    const int line = 128 / static_cast<int>(c->elem());  // elements per cache line
    c->pitch = (nx + line - 1) / line * line;
  }
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDevice");
  }
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "hipStreamCreateWithFlags");
    }
    c->own_stream = true;
  }
  const size_t N = c->plane_elems();
  qla_status st = QLA_OK;
  for (int b = 0; b < 2 && st == QLA_OK; ++b)
    for (int k = 0; k < 3 && st == QLA_OK; ++k) st = alloc(&c->q[b][k], N * c->elem(), "amplitudes");
  if (st == QLA_OK) st = alloc(reinterpret_cast<void**>(&c->n64), N * sizeof(double), "index");
  if (st == QLA_OK && c->fp32)
    st = alloc(reinterpret_cast<void**>(&c->n32), N * sizeof(float), "index fp32");
  if (st == QLA_OK)
    st = alloc(reinterpret_cast<void**>(&c->staging), 3 * N * sizeof(double), "staging");
  if (st == QLA_OK)
    st = alloc(reinterpret_cast<void**>(&c->partials),
               3 * qla::kEnergyPartials * sizeof(double), "partials");
  if (st == QLA_OK) st = alloc(reinterpret_cast<void**>(&c->diag), 3 * sizeof(double), "diag");
  if (st == QLA_OK) st = alloc(reinterpret_cast<void**>(&c->energy_dev), sizeof(double), "energy");
  if (st == QLA_OK)
    st = alloc(reinterpret_cast<void**>(&c->stats), 4 * sizeof(unsigned long long), "stats");
  if (st == QLA_OK) {
    for (int k = 0; k < 3 && st == QLA_OK; ++k) {
      e = hipMemsetAsync(c->q[0][k], 0, N * c->elem(), c->stream);
      if (e != hipSuccess) st = hip_fail(e, "hipMemsetAsync");
    }
    if (st == QLA_OK) {
      e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
  }
  if (st != QLA_OK) {
    release(c);
    delete c;
    return st;
  }
  *out = c;
  return QLA_OK;
}

qla_status qla_destroy(qla_ctx* c) {
  if (!c) return QLA_OK;
  if (c->owned_by_batch) return fail(QLA_EINVAL, "this context belongs to a batch");
  DeviceGuard g(c->device);  // frees what it can even if selecting the device fails
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  release(c);
  delete c;
  return QLA_OK;
}

qla_status qla_set_index(qla_ctx* c, const double* n_host, size_t ld) {
  if (!c || !n_host) return fail(QLA_EINVAL, "NULL argument");
  if (ld < static_cast<size_t>(c->nx)) return fail(QLA_EINVAL, "ld < nx");
  QLA_ON_DEVICE(c->device);
  // raw rows into the first staging plane (packed), then validate from there; a blocking
  // copy once the stream is idle (nothing queued still reads the staging planes)
  QLA_HIP(hipStreamSynchronize(c->stream));
  QLA_HIP(hipMemcpy2D(c->staging, c->nx * sizeof(double), n_host, ld * sizeof(double),
                      c->nx * sizeof(double), c->ny, hipMemcpyHostToDevice));
  return install_index(c, c->staging, c->nx);
}

qla_status qla_set_index_ellipse(qla_ctx* c, const qla_ellipse* e) {
  if (!c || !e) return fail(QLA_EINVAL, "NULL argument");
  const double v[] = {e->xc, e->yc, e->a, e->b, e->rot, e->n_in, e->n_out, e->width};
  for (double x : v)
    if (!std::isfinite(x)) return fail(QLA_EINVAL, "ellipse: every field must be finite");
  if (!(e->a > 0.0) || !(e->b > 0.0) || !(e->width > 0.0))
    return fail(QLA_EINVAL, "ellipse: a, b and width must be > 0");
  QLA_ON_DEVICE(c->device);
  const qla::EllipseArgs a{e->xc, e->yc, e->a, e->b, e->rot, e->n_in, e->n_out, e->width};
  QLA_HIP(qla::launch_ellipse_index(c->nx, c->ny, a, c->staging, c->stream));
  return install_index(c, c->staging, c->nx);
}

qla_status qla_set_index_device(qla_ctx* c, const double* n_device, size_t ld) {
  if (!c || !n_device) return fail(QLA_EINVAL, "NULL argument");
  if (ld < static_cast<size_t>(c->nx)) return fail(QLA_EINVAL, "ld < nx");
  QLA_ON_DEVICE(c->device);
  return install_index(c, n_device, ld);
}

qla_status qla_init_packet(qla_ctx* c, const qla_packet* p) {
  if (!c || !p) return fail(QLA_EINVAL, "NULL argument");
  if (!c->have_index) return fail(QLA_ESTATE, "set the refractive index first");
  if (!(p->sigma > 0.0) || !(p->lambda > 0.0) || !std::isfinite(p->x0) || !std::isfinite(p->y0) ||
      !std::isfinite(p->phi) || !std::isfinite(p->amp) || !std::isfinite(p->sigma) ||
      !std::isfinite(p->lambda))
    return fail(QLA_EINVAL, "packet: sigma and lambda must be > 0 and all fields finite");
  QLA_ON_DEVICE(c->device);
  qla::PacketArgs a{p->x0, p->y0, p->sigma, p->lambda, p->phi, p->amp, p->planar, c->triple};
  QLA_HIP(qla::launch_packet(c->n64, c->nx, c->ny, c->pitch, a, c->fp32, c->q[c->cur][0],
                             c->q[c->cur][1], c->q[c->cur][2], c->stream));
  c->steps = 0;
  return QLA_OK;
}

qla_status qla_set_fields(qla_ctx* c, const double* q_host, int64_t step) {
  if (!c || !q_host) return fail(QLA_EINVAL, "NULL argument");
  if (step < 0) return fail(QLA_EINVAL, "step < 0");
  QLA_ON_DEVICE(c->device);
  const size_t N = c->count();
  QLA_HIP(hipStreamSynchronize(c->stream));
  QLA_HIP(hipMemcpy(c->staging, q_host, 3 * N * sizeof(double), hipMemcpyHostToDevice));
  QLA_HIP(qla::launch_from_f64(c->staging, c->nx, c->ny, c->pitch, c->fp32,
                               c->q[c->cur][c->plane(0)],
                               c->q[c->cur][c->plane(1)], c->q[c->cur][c->plane(2)], c->stream));
  QLA_HIP(hipStreamSynchronize(c->stream));
  c->steps = step;
  return QLA_OK;
}


qla_status qla_advance(qla_ctx* c, int64_t k) {
  if (!c) return fail(QLA_EINVAL, "NULL context");
  if (k < 0) return fail(QLA_EINVAL, "k < 0");
  if (!c->have_index) return fail(QLA_ESTATE, "set the refractive index first");
  QLA_ON_DEVICE(c->device);
  return enqueue_steps(c, k, c->rows_per_seg, c->prefetch, c->fused, c->cols);
}

qla_status qla_autotune(qla_ctx* c, int* rows_out, int* prefetch_out, int* steps_per_pass_out) {
  if (!c) return fail(QLA_EINVAL, "NULL context");
  if (!c->have_index) return fail(QLA_ESTATE, "set the refractive index first");
  QLA_ON_DEVICE(c->device);
  // keep the state: the trial launches overwrite both amplitude buffers
  const size_t plane_bytes = c->plane_elems() * c->elem();
  char* save = reinterpret_cast<char*>(c->staging);
  for (int j = 0; j < 3; ++j)
    QLA_HIP(hipMemcpyAsync(save + j * plane_bytes, c->q[c->cur][j], plane_bytes,
                           hipMemcpyDeviceToDevice, c->stream));
  const int64_t steps_saved = c->steps;
  const int cur_saved = c->cur;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  QLA_HIP(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(he, "hipEventCreate");
  }
  static const int kRows[] = {24, 40, 56, 80, 112, 144, 176, 240, 320, 480, 720};
  static const int kPrefetch[] = {2, 3};
  static const int kFused[] = {1, 2};
  // two columns per lane only where the kernel has them (FP32, even width)
  const int max_cols = (c->fp32 && c->nx % 2 == 0) ? 2 : 1;
  // Each trial times enough steps for about 4e8 site updates (a few milliseconds; at
  // least 8, even), after a warm-up of the same length that brings the clocks up. The
  // four fastest candidates of the sweep are timed twice more and the best time of
  // each counts, so one noisy trial does not decide the tuning.
  const double sites = static_cast<double>(c->count());
  int64_t trial = static_cast<int64_t>(std::ceil(4e8 / sites));
  trial = std::min<int64_t>(512, std::max<int64_t>(8, trial + (trial & 1)));
  struct Cand {
    double per_step;
    int rows, pf, fused, cols;
  };
  qla_status st = QLA_OK;
  auto time_one = [&](const Cand& k, double* per_step) -> qla_status {
    qla_status s2 = enqueue_steps(c, k.fused, k.rows, k.pf, k.fused, k.cols);  // warm pass
    if (s2 != QLA_OK) return s2;
    hipError_t h = hipEventRecord(e0, c->stream);
    if (h == hipSuccess) s2 = enqueue_steps(c, trial, k.rows, k.pf, k.fused, k.cols);
    if (h == hipSuccess && s2 == QLA_OK) h = hipEventRecord(e1, c->stream);
    if (h == hipSuccess && s2 == QLA_OK) h = hipEventSynchronize(e1);
    float ms = 0.f;
    if (h == hipSuccess && s2 == QLA_OK) h = hipEventElapsedTime(&ms, e0, e1);
    if (h != hipSuccess) return hip_fail(h, "autotune timing");
    if (s2 != QLA_OK) return s2;
    *per_step = ms / static_cast<double>(trial);
    return QLA_OK;
  };
  st = enqueue_steps(c, trial, c->rows_per_seg, c->prefetch, c->fused, c->cols);  // warm-up
  std::vector<Cand> cands;
  for (int cols = 1; cols <= max_cols; ++cols)
    for (int fused : kFused)
      for (int pf : kPrefetch)
        for (int rows : kRows) {
          if (rows > c->ny + 8 && rows != kRows[0]) continue;
          cands.push_back({0.0, rows, pf, fused, cols});
        }
  for (size_t k = 0; k < cands.size() && st == QLA_OK; ++k)
    st = time_one(cands[k], &cands[k].per_step);
  if (st == QLA_OK) {
    std::sort(cands.begin(), cands.end(),
              [](const Cand& a, const Cand& b) { return a.per_step < b.per_step; });
    const size_t top = std::min<size_t>(4, cands.size());
    for (int rep = 0; rep < 2 && st == QLA_OK; ++rep)
      for (size_t k = 0; k < top && st == QLA_OK; ++k) {
        double t = 0.0;
        st = time_one(cands[k], &t);
        cands[k].per_step = std::min(cands[k].per_step, t);
      }
    std::sort(cands.begin(), cands.begin() + top,
              [](const Cand& a, const Cand& b) { return a.per_step < b.per_step; });
    // Among the candidates within 3% of the fastest, take the one that recomputes the
    // fewest halo sites. Trials can rank near-equal candidates differently from long
    // runs (16384^2 FP64: 56-row segments won the trials, 112-row ones ran 8% faster
    // over 20000 steps), and less redundant arithmetic is the safer choice.
    auto redundancy = [&](const Cand& k) {
      const int win = k.pf + 4 * k.fused + 2, halo = 4 * k.fused;
      const int rows = ((k.rows + 2 * halo + win - 1) / win) * win - 2 * halo;
      const double wide = 64.0 * k.cols;
      return (rows + 2.0 * halo) / rows * wide / (wide - 2.0 * halo);
    };
    size_t pick = 0;
    for (size_t k = 1; k < top; ++k)
      if (cands[k].per_step <= 1.03 * cands[0].per_step &&
          redundancy(cands[k]) < redundancy(cands[pick]))
        pick = k;
    std::swap(cands[0], cands[pick]);
  }
  int brows = c->rows_per_seg, bpf = c->prefetch, bfused = c->fused, bcols = c->cols;
  if (st == QLA_OK && !cands.empty()) {
    brows = cands[0].rows;
    bpf = cands[0].pf;
    bfused = cands[0].fused;
    bcols = cands[0].cols;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->cur = cur_saved;
  c->steps = steps_saved;
  for (int j = 0; j < 3; ++j)
    QLA_HIP(hipMemcpyAsync(c->q[c->cur][j], save + j * plane_bytes, plane_bytes,
                           hipMemcpyDeviceToDevice, c->stream));
  QLA_HIP(hipStreamSynchronize(c->stream));
  if (st != QLA_OK) return st;
  c->rows_per_seg = brows;
  c->prefetch = bpf;
  c->fused = bfused;
  c->cols = bcols;
  if (rows_out) *rows_out = brows;
  if (prefetch_out) *prefetch_out = bpf;
  if (steps_per_pass_out) *steps_per_pass_out = bfused;
  return QLA_OK;
}

qla_status qla_get_tuning(const qla_ctx* c, int* rows, int* prefetch, int* steps_per_pass) {
  if (!c) return fail(QLA_EINVAL, "NULL context");
  if (rows) *rows = c->rows_per_seg;
  if (prefetch) *prefetch = c->prefetch;
  if (steps_per_pass) *steps_per_pass = c->fused;
  return QLA_OK;
}

qla_status qla_get_fields_device(qla_ctx* c, double* out, int physical) {
  if (!c || !out) return fail(QLA_EINVAL, "NULL argument");
  if (physical && !c->have_index) return fail(QLA_ESTATE, "physical readout needs the index");
  QLA_ON_DEVICE(c->device);
  QLA_HIP(qla::launch_readout(c->q[c->cur][c->plane(0)], c->q[c->cur][c->plane(1)],
                              c->q[c->cur][c->plane(2)], c->n64, c->nx, c->ny, c->pitch,
                              c->fp32, divide_mask(c, physical), out, c->stream));
  return QLA_OK;
}

qla_status qla_get_fields(qla_ctx* c, double* out_host, int physical) {
  if (!c || !out_host) return fail(QLA_EINVAL, "NULL argument");
  if (physical && !c->have_index) return fail(QLA_ESTATE, "physical readout needs the index");
  QLA_ON_DEVICE(c->device);
  QLA_HIP(qla::launch_readout(c->q[c->cur][c->plane(0)], c->q[c->cur][c->plane(1)],
                              c->q[c->cur][c->plane(2)], c->n64, c->nx, c->ny, c->pitch,
                              c->fp32, divide_mask(c, physical), c->staging, c->stream));
  QLA_HIP(hipMemcpyAsync(out_host, c->staging, 3 * c->count() * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  QLA_HIP(hipStreamSynchronize(c->stream));
  return QLA_OK;
}

qla_status qla_energy_device(qla_ctx* c, double* energy_device) {
  if (!c || !energy_device) return fail(QLA_EINVAL, "NULL argument");
  QLA_ON_DEVICE(c->device);
  QLA_HIP(qla::launch_energy(c->q[c->cur][0], c->q[c->cur][1], c->q[c->cur][2], c->nx, c->ny,
                             c->pitch, c->fp32, c->partials, energy_device, c->stream));
  return QLA_OK;
}

qla_status qla_energy(qla_ctx* c, double* energy) {
  if (!c || !energy) return fail(QLA_EINVAL, "NULL argument");
  QLA_ON_DEVICE(c->device);
  QLA_HIP(qla::launch_energy(c->q[c->cur][0], c->q[c->cur][1], c->q[c->cur][2], c->nx, c->ny,
                             c->pitch, c->fp32, c->partials, c->energy_dev, c->stream));
  QLA_HIP(hipMemcpyAsync(energy, c->energy_dev, sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  QLA_HIP(hipStreamSynchronize(c->stream));
  return QLA_OK;
}

qla_status qla_divergence(qla_ctx* c, double* l2, double* max_abs, double* scale) {
  if (!c) return fail(QLA_EINVAL, "NULL context");
  if (c->triple == 1 && !c->have_index)
    return fail(QLA_ESTATE, "the B_z triple's divergence (of D = n^2 E) needs the index");
  QLA_ON_DEVICE(c->device);
  // stored planes (shared, y partner, x partner) = (q2, q3, q4) or (q5, q0, q1): the
  // in-plane field is (stored 1, stored 2), i.e. (Bx, By) or (n Ex, n Ey)
  QLA_HIP(qla::launch_divergence(c->q[c->cur][1], c->q[c->cur][2], c->n64, c->nx, c->ny,
                                 c->pitch, c->delta, c->fp32, c->triple == 1, c->partials, c->diag,
                                 c->stream));
  double h[3];
  QLA_HIP(hipMemcpyAsync(h, c->diag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  QLA_HIP(hipStreamSynchronize(c->stream));
  if (l2) *l2 = std::sqrt(h[0]);
  if (max_abs) *max_abs = h[1];
  if (scale) *scale = std::sqrt(h[2]);
  return QLA_OK;
}

qla_status qla_get_coefficients(qla_ctx* c, double* theta, double* beta_x, double* beta_y) {
  if (!c) return fail(QLA_EINVAL, "NULL context");
  if (!c->have_index) return fail(QLA_ESTATE, "set the refractive index first");
  QLA_ON_DEVICE(c->device);
  const size_t N = c->count();
  double* s = c->staging;
  QLA_HIP(qla::launch_coefficients(c->n64, c->nx, c->ny, c->pitch, c->delta, s, s + N,
                                   s + 2 * N, c->stream));
  double* dst[3] = {theta, beta_x, beta_y};
  for (int k = 0; k < 3; ++k)
    if (dst[k])
      QLA_HIP(hipMemcpyAsync(dst[k], s + k * N, N * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  QLA_HIP(hipStreamSynchronize(c->stream));
  return QLA_OK;
}

qla_status qla_step_count(const qla_ctx* c, int64_t* steps) {
  if (!c || !steps) return fail(QLA_EINVAL, "NULL argument");
  *steps = c->steps;
  return QLA_OK;
}

qla_status qla_set_tuning(qla_ctx* c, int rows_per_segment, int prefetch_rows,
                          int steps_per_pass) {
  if (!c) return fail(QLA_EINVAL, "NULL context");
  if (rows_per_segment < 0 || rows_per_segment > (1 << 20))
    return fail(QLA_EINVAL, "rows_per_segment must be in [0, 2^20]");
  if (prefetch_rows != 0 && prefetch_rows != 2 && prefetch_rows != 3)
    return fail(QLA_EINVAL, "prefetch_rows must be 0 (default), 2 or 3");
  if (steps_per_pass < 0 || steps_per_pass > 2)
    return fail(QLA_EINVAL, "steps_per_pass must be 0 (default), 1 or 2");
  c->rows_per_seg = rows_per_segment ? rows_per_segment : qla::kDefaultRows;
  c->prefetch = prefetch_rows ? prefetch_rows : qla::kDefaultPrefetch;
  c->fused = steps_per_pass ? steps_per_pass : qla::kDefaultFused;
  return QLA_OK;
}

qla_status qla_set_lane_columns(qla_ctx* c, int columns) {
  if (!c) return fail(QLA_EINVAL, "NULL context");
  if (columns < 0 || columns > 2) return fail(QLA_EINVAL, "columns must be 0 (default), 1 or 2");
  if (columns == 2 && !c->fp32) return fail(QLA_EINVAL, "two columns per lane need FP32");
  if (columns == 2 && c->nx % 2 != 0) return fail(QLA_EINVAL, "two columns per lane need even nx");
  c->cols = columns ? columns : 1;
  return QLA_OK;
}

qla_status qla_get_lane_columns(const qla_ctx* c, int* columns) {
  if (!c || !columns) return fail(QLA_EINVAL, "NULL argument");
  *columns = c->cols;
  return QLA_OK;
}

}  // extern "C"
