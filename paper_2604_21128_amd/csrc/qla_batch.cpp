// Batched C ABI (include/qla.h, qla_batch_*): many independent lattices of uneven
// sizes advanced together. Every pass is one persistent launch that strides over
// the wavefront tiles of all lattices still running; the passes of a whole run are
// captured once into a hipGraph and replayed by qla_batch_run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "qla.h"
#include "qla_ctx.h"
#include "qla_internal.h"

using qla::DeviceGuard;
using qla::fail;
using qla::hip_fail;

struct qla_batch {
  int count = 0;
  bool fp32 = false;
  int vmode = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<qla_ctx*> ctx;
  // plan
  bool planned = false;
  std::vector<int64_t> steps;
  int rows = 0, prefetch = 0, fused = 0, mode = 0, passes = 0, angle_class = 0, blocks = 0;
  bool fit = false;               // segment heights fitted per lattice around `rows`
  int64_t total_updates = 0;
  void* d_args = nullptr;
  unsigned* d_items = nullptr;
  int* d_counts = nullptr;
  int* d_parity = nullptr;        // per instance, see qla_batch_kernel
  std::vector<int> parity;        // host copy
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kMaxInstances = 4095;  // instance index field of an item: 12 bits
constexpr int kMaxTiles = 1 << 20;   // tile index field: 20 bits

void release_plan(qla_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_args) (void)hipFree(b->d_args);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_counts) (void)hipFree(b->d_counts);
  if (b->d_parity) (void)hipFree(b->d_parity);
  b->d_parity = nullptr;
  b->exec = nullptr;
  b->graph = nullptr;
  b->d_args = nullptr;
  b->d_items = nullptr;
  b->d_counts = nullptr;
  b->planned = false;
}

struct Tables {
  std::vector<char> args;       // 2 StepArgs per instance
  std::vector<unsigned> items;  // (instance << 20 | tile), instances by decreasing passes
  std::vector<int> counts;      // items of the instances still running, per pass
  int passes = 0;
};

// Segment height for one lattice of ny rows. A wavefront marches whole unrolled loop
// trips of `win` rows (the register window), so the heights it can realise are
// win k - 2 halo; among those from 3/4 to 3/2 of the target, take the one that
// covers ny with the fewest marched rows (segments x trips x win), ties to the
// height closest to the target. A lattice of 300 rows with a 62-row target then
// takes four 75-row segments (364 marched rows) instead of five of 62 (390).
int fitted_rows(int ny, int target, int prefetch, int fused) {
  const int win = prefetch + 4 * fused + 2, halo = 4 * fused;
  int best = target;
  int64_t best_cost = INT64_MAX;
  for (int k = 1; win * k - 2 * halo <= (3 * target) / 2 || k == 1; ++k) {
    const int rows = win * k - 2 * halo;
    if (rows < 1 || 4 * rows < 3 * target) continue;
    const int64_t cost = static_cast<int64_t>((ny + rows - 1) / rows) * win * k;
    if (cost < best_cost ||
        (cost == best_cost && std::abs(rows - target) < std::abs(best - target))) {
      best_cost = cost;
      best = rows;
    }
  }
  return best;
}

// Builds the launch tables for one tuning (segment height `rows` for every lattice,
// or fitted to each lattice's height around it). Returns false if a lattice has
// more tiles than an item can address.
bool build_tables(const qla_batch* b, int rows, int prefetch, int fused, bool fit,
                  Tables* t) {
  const size_t asz = qla::step_args_bytes(b->fp32);
  t->args.assign(2 * b->count * asz, 0);
  std::vector<int> tiles(b->count), passes(b->count);
  for (int i = 0; i < b->count; ++i) {
    const int r = fit ? fitted_rows(b->ctx[i]->ny, rows, prefetch, fused) : rows;
    for (int dir = 0; dir < 2; ++dir) {
      const qla::StepLaunch L = qla::step_launch_for(b->ctx[i], r, prefetch, fused, dir);
      qla::fill_step_args(L, t->args.data() + (2 * i + dir) * asz, &tiles[i]);
    }
    if (tiles[i] > kMaxTiles) return false;
    passes[i] = static_cast<int>(b->steps[i] / fused);
  }
  std::vector<int> order(b->count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return passes[x] != passes[y] ? passes[x] > passes[y] : tiles[x] > tiles[y];
  });
  t->passes = b->count ? passes[order[0]] : 0;
  t->items.clear();
  std::vector<int> end_of(b->count);
  for (int i : order) {
    for (int k = 0; k < tiles[i]; ++k)
      t->items.push_back((static_cast<unsigned>(i) << 20) | static_cast<unsigned>(k));
    end_of[i] = static_cast<int>(t->items.size());
  }
  t->counts.assign(t->passes, 0);
  for (int p = 0; p < t->passes; ++p) {
    int n = 0;
    for (int i : order)
      if (passes[i] > p) n = end_of[i];
    t->counts[p] = n;
  }
  return true;
}

qla_status upload(qla_batch* b, const Tables& t, void** d_args, unsigned** d_items,
                  int** d_counts) {
  *d_args = nullptr;
  *d_items = nullptr;
  *d_counts = nullptr;
  hipError_t e = hipMalloc(d_args, t.args.size());
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(d_items),
                                     std::max<size_t>(1, t.items.size()) * sizeof(unsigned));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(d_counts),
                                     std::max<size_t>(1, t.counts.size()) * sizeof(int));
  if (e != hipSuccess) {
    if (*d_args) (void)hipFree(*d_args);
    if (*d_items) (void)hipFree(*d_items);
    if (*d_counts) (void)hipFree(*d_counts);
    *d_args = nullptr;
    *d_items = nullptr;
    *d_counts = nullptr;
    return fail(QLA_ENOMEM, std::string("batch tables: ") + hipGetErrorString(e));
  }
  QLA_HIP(hipMemcpyAsync(*d_args, t.args.data(), t.args.size(), hipMemcpyHostToDevice,
                         b->stream));
  if (!t.items.empty())
    QLA_HIP(hipMemcpyAsync(*d_items, t.items.data(), t.items.size() * sizeof(unsigned),
                           hipMemcpyHostToDevice, b->stream));
  if (!t.counts.empty())
    QLA_HIP(hipMemcpyAsync(*d_counts, t.counts.data(), t.counts.size() * sizeof(int),
                           hipMemcpyHostToDevice, b->stream));
  return QLA_OK;
}

qla::BatchLaunch batch_launch(const qla_batch* b, const void* args, const unsigned* items,
                              const int* counts, const int* parity, int prefetch, int fused) {
  qla::BatchLaunch B{};
  B.args = args;
  B.items = items;
  B.counts = counts;
  B.parity = parity;
  B.fp32 = b->fp32;
  B.vmode = b->vmode;
  B.angle_class = b->angle_class;
  B.prefetch = prefetch;
  B.fused = fused;
  return B;
}

// Enqueues passes [p0, p1), one launch each.
qla_status enqueue_passes(qla_batch* b, qla::BatchLaunch B, int p0, int p1) {
  for (int p = p0; p < p1; ++p) {
    B.pass = p;
    QLA_HIP(qla::launch_batch(B, b->stream));
  }
  return QLA_OK;
}

qla_status save_states(qla_batch* b) {
  for (qla_ctx* c : b->ctx)
    for (int j = 0; j < 3; ++j)
      QLA_HIP(hipMemcpyAsync(reinterpret_cast<char*>(c->staging) + j * c->plane_elems() * c->elem(),
                             c->q[c->cur][j], c->plane_elems() * c->elem(), hipMemcpyDeviceToDevice,
                             b->stream));
  return QLA_OK;
}

qla_status restore_states(qla_batch* b) {
  for (qla_ctx* c : b->ctx)
    for (int j = 0; j < 3; ++j)
      QLA_HIP(hipMemcpyAsync(c->q[c->cur][j],
                             reinterpret_cast<char*>(c->staging) + j * c->plane_elems() * c->elem(),
                             c->plane_elems() * c->elem(), hipMemcpyDeviceToDevice, b->stream));
  return QLA_OK;
}

// Time a few passes of the batch under one tuning; returns ns per lattice-site update.
qla_status time_candidate(qla_batch* b, int rows, int prefetch, int fused, bool fit,
                          double* ns_per_update) {
  *ns_per_update = 1e300;
  Tables t;
  if (!build_tables(b, rows, prefetch, fused, fit, &t)) return QLA_OK;
  void* d_args;
  unsigned* d_items;
  int* d_counts;
  qla_status st = upload(b, t, &d_args, &d_items, &d_counts);
  if (st != QLA_OK) return st;
  qla::BatchLaunch B = batch_launch(b, d_args, d_items, d_counts, b->d_parity, prefetch, fused);
  hipError_t e = qla::batch_resident_blocks(B, &B.blocks);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int trial = std::min(t.passes, 3);
  if (e == hipSuccess && trial > 0) {
    // warm-up pass, then the timed passes (pass parity does not matter for timing:
    // the buffers' contents are restored afterwards)
    st = enqueue_passes(b, B, 0, 1);
    if (st == QLA_OK) e = hipEventRecord(e0, b->stream);
    if (st == QLA_OK && e == hipSuccess) st = enqueue_passes(b, B, 0, trial);
    if (st == QLA_OK && e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (st == QLA_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (st == QLA_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (st == QLA_OK && e == hipSuccess) {
      double updates = 0.0;
      for (int i = 0; i < b->count; ++i)
        if (b->steps[i] / fused > 0)
          updates += static_cast<double>(b->ctx[i]->count()) * fused *
                     std::min<int64_t>(trial, b->steps[i] / fused);
      *ns_per_update = ms * 1e6 / updates;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(b->stream);
  (void)hipFree(d_args);
  (void)hipFree(d_items);
  (void)hipFree(d_counts);
  if (st != QLA_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "batch timing");
  return QLA_OK;
}

}  // namespace

extern "C" {

qla_status qla_batch_create(int count, const int* nx, const int* ny, const double* delta,
                            qla_precision precision, qla_potential potential, void* hip_stream,
                            qla_batch** out) {
  if (!out) return fail(QLA_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || count > kMaxInstances)
    return fail(QLA_EINVAL, "count must be in [1, " + std::to_string(kMaxInstances) + "]");
  if (!nx || !ny || !delta) return fail(QLA_EINVAL, "NULL size array");
  qla_batch* b = new (std::nothrow) qla_batch;
  if (!b) return fail(QLA_ENOMEM, "host allocation");
  b->count = count;
  b->fp32 = precision == QLA_F32;
  b->vmode = static_cast<int>(potential);
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDevice");
  }
  if (hip_stream) {
    b->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete b;
      return hip_fail(e, "hipStreamCreateWithFlags");
    }
    b->own_stream = true;
  }
  for (int i = 0; i < count; ++i) {
    // the batched kernel addresses each plane through one buffer descriptor (rows padded
    // to whole 128-byte lines)
    const long long elem = b->fp32 ? 4 : 8, line = 128 / elem;
    const long long bytes = (nx[i] + line - 1) / line * line * ny[i] * elem;
    if (bytes > (1ll << 31)) {
      if (b->own_stream) (void)hipStreamDestroy(b->stream);
      delete b;
      return fail(QLA_EINVAL, "instance " + std::to_string(i) +
                                  ": a batched lattice's plane must fit in 2 GiB");
    }
  }
  b->ctx.assign(count, nullptr);
  for (int i = 0; i < count; ++i) {
    const qla_status st = qla_create(nx[i], ny[i], delta[i], precision, potential, b->stream,
                                     &b->ctx[i]);
    if (st != QLA_OK) {
      const std::string msg = "instance " + std::to_string(i) + ": " + qla_last_error();
      for (int j = 0; j < i; ++j) qla_destroy(b->ctx[j]);
      if (b->own_stream) (void)hipStreamDestroy(b->stream);
      delete b;
      return fail(st, msg);
    }
    b->ctx[i]->owned_by_batch = true;
  }
  *out = b;
  return QLA_OK;
}

qla_status qla_batch_context(qla_batch* b, int i, qla_ctx** ctx) {
  if (!b || !ctx) return fail(QLA_EINVAL, "NULL argument");
  if (i < 0 || i >= b->count) return fail(QLA_EINVAL, "instance index out of range");
  *ctx = b->ctx[i];
  return QLA_OK;
}

}  // extern "C"

namespace {

struct BatchTuning {
  int rows, prefetch, fused;
  bool fit;
};

// Plans the run: with `fixed` NULL the tuning is autotuned on the batch itself.
qla_status plan_batch(qla_batch* b, const int64_t* steps, const BatchTuning* fixed) {
  bool all_even = true;
  int cls = 0;
  for (int i = 0; i < b->count; ++i) {
    if (steps[i] < 0) return fail(QLA_EINVAL, "steps must be >= 0");
    if (!b->ctx[i]->have_index)
      return fail(QLA_ESTATE, "instance " + std::to_string(i) + " has no index");
    all_even = all_even && (steps[i] % 2 == 0);
    cls = std::max(cls, b->ctx[i]->angle_class);
  }
  if (fixed && fixed->fused == 2 && !all_even)
    return fail(QLA_EINVAL, "two steps per pass need an even step count for every lattice");
  QLA_ON_DEVICE(b->device);
  release_plan(b);
  b->steps.assign(steps, steps + b->count);
  b->angle_class = cls;
  // the tables are built from each lattice's current buffer: no swap yet
  b->parity.assign(b->count, 0);
  {
    const hipError_t pe = hipMalloc(reinterpret_cast<void**>(&b->d_parity),
                                    b->count * sizeof(int));
    if (pe != hipSuccess) {
      b->d_parity = nullptr;
      return fail(QLA_ENOMEM, std::string("batch parity: ") + hipGetErrorString(pe));
    }
    QLA_HIP(hipMemcpyAsync(b->d_parity, b->parity.data(), b->count * sizeof(int),
                           hipMemcpyHostToDevice, b->stream));
  }
  // --- tuning, given or autotuned: tile height (one for all lattices, or fitted to
  // each lattice's height around it), prefetch depth and steps per pass
  static const int kRows[] = {24, 56, 88, 152};
  static const int kPrefetch[] = {2, 3};
  const int fused_options[2] = {all_even ? 2 : 1, 1};
  const int n_fused = all_even ? 2 : 1;
  int brows = qla::kDefaultRows, bpf = qla::kDefaultPrefetch, bfused = fused_options[0];
  bool bfit = false;
  const int bmode = 1;
  qla_status st = QLA_OK;
  if (fixed) {
    brows = fixed->rows;
    bpf = fixed->prefetch;
    bfused = fixed->fused;
    bfit = fixed->fit;
  } else {
    st = save_states(b);
    if (st != QLA_OK) return st;
    double best = 1e300;
    for (int fi = 0; fi < n_fused && st == QLA_OK; ++fi) {
      for (int pf : kPrefetch) {
        for (int rows : kRows) {
          for (int fit = 0; fit < 2 && st == QLA_OK; ++fit) {
            double ns = 1e300;
            st = time_candidate(b, rows, pf, fused_options[fi], fit != 0, &ns);
            if (st == QLA_OK && ns < best) {
              best = ns;
              brows = rows;
              bpf = pf;
              bfused = fused_options[fi];
              bfit = fit != 0;
            }
          }
          if (st != QLA_OK) break;
        }
        if (st != QLA_OK) break;
      }
    }
    const qla_status rs = restore_states(b);
    if (st != QLA_OK) return st;
    if (rs != QLA_OK) return rs;
  }
  // --- tables and graph for the chosen tuning
  Tables t;
  if (!build_tables(b, brows, bpf, bfused, bfit, &t))
    return fail(QLA_EINVAL, "a lattice has more than 2^20 wavefront tiles");
  st = upload(b, t, &b->d_args, &b->d_items, &b->d_counts);
  if (st != QLA_OK) return st;
  qla::BatchLaunch B =
      batch_launch(b, b->d_args, b->d_items, b->d_counts, b->d_parity, bpf, bfused);
  QLA_HIP(qla::batch_resident_blocks(B, &B.blocks));
  QLA_HIP(hipStreamSynchronize(b->stream));
  QLA_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  st = enqueue_passes(b, B, 0, t.passes);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(b->stream, &graph);
  if (st != QLA_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
  b->graph = graph;
  QLA_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->rows = brows;
  b->fit = bfit;
  b->prefetch = bpf;
  b->fused = bfused;
  b->mode = bmode;
  b->passes = t.passes;
  b->blocks = B.blocks;
  b->total_updates = 0;
  for (int i = 0; i < b->count; ++i)
    b->total_updates += static_cast<int64_t>(b->ctx[i]->count()) * (steps[i] / bfused) * bfused;
  b->planned = true;
  return QLA_OK;
}

}  // namespace

extern "C" {

qla_status qla_batch_plan(qla_batch* b, const int64_t* steps, int mode) {
  if (!b || !steps) return fail(QLA_EINVAL, "NULL argument");
  if (mode == 2)
    return fail(QLA_EINVAL, "mode 2 (one cooperative launch per run) is not available; "
                            "use 0 or 1");
  if (mode < 0 || mode > 1) return fail(QLA_EINVAL, "mode must be 0 (auto) or 1");
  return plan_batch(b, steps, nullptr);
}

qla_status qla_batch_plan_fixed(qla_batch* b, const int64_t* steps, int rows_per_segment,
                                int prefetch_rows, int steps_per_pass, int fit) {
  if (!b || !steps) return fail(QLA_EINVAL, "NULL argument");
  if (rows_per_segment < 1 || rows_per_segment > (1 << 20))
    return fail(QLA_EINVAL, "rows_per_segment must be in [1, 2^20]");
  if (prefetch_rows != 2 && prefetch_rows != 3)
    return fail(QLA_EINVAL, "prefetch_rows must be 2 or 3");
  if (steps_per_pass != 1 && steps_per_pass != 2)
    return fail(QLA_EINVAL, "steps_per_pass must be 1 or 2");
  if (fit != 0 && fit != 1) return fail(QLA_EINVAL, "fit must be 0 or 1");
  const BatchTuning t{rows_per_segment, prefetch_rows, steps_per_pass, fit != 0};
  return plan_batch(b, steps, &t);
}

qla_status qla_batch_run(qla_batch* b) {
  if (!b) return fail(QLA_EINVAL, "NULL batch");
  if (!b->planned) return fail(QLA_ESTATE, "plan the batch first");
  // The captured launches evaluate the rotation angles with the series length of the
  // indices set when the run was planned; an index set since then with larger angles
  // needs the longer series, so the run must be planned again.
  for (int i = 0; i < b->count; ++i)
    if (b->ctx[i]->angle_class > b->angle_class)
      return fail(QLA_ESTATE, "instance " + std::to_string(i) +
                                  ": its index was set after planning and has angles beyond "
                                  "the planned run's range; plan the batch again");
  QLA_ON_DEVICE(b->device);
  QLA_HIP(hipGraphLaunch(b->exec, b->stream));
  // An odd number of passes leaves a lattice's result in its other buffer: its
  // context follows, and its parity flips for the next run of the same graph.
  bool flipped = false;
  for (int i = 0; i < b->count; ++i) {
    const int64_t passes = b->steps[i] / b->fused;
    if (passes & 1) {
      b->ctx[i]->cur ^= 1;
      b->parity[i] ^= 1;
      flipped = true;
    }
    b->ctx[i]->steps += passes * b->fused;
  }
  if (flipped)
    QLA_HIP(hipMemcpyAsync(b->d_parity, b->parity.data(), b->count * sizeof(int),
                           hipMemcpyHostToDevice, b->stream));
  return QLA_OK;
}

qla_status qla_batch_plan_info(const qla_batch* b, int* rows, int* prefetch, int* steps_per_pass,
                               int* mode, int* passes, int64_t* site_updates) {
  if (!b) return fail(QLA_EINVAL, "NULL batch");
  if (!b->planned) return fail(QLA_ESTATE, "the batch is not planned");
  if (rows) *rows = b->rows;
  if (prefetch) *prefetch = b->prefetch;
  if (steps_per_pass) *steps_per_pass = b->fused;
  if (mode) *mode = b->mode;
  if (passes) *passes = b->passes;
  if (site_updates) *site_updates = b->total_updates;
  return QLA_OK;
}

qla_status qla_batch_segment_rows(const qla_batch* b, int i, int* rows) {
  if (!b || !rows) return fail(QLA_EINVAL, "NULL argument");
  if (!b->planned) return fail(QLA_ESTATE, "the batch is not planned");
  if (i < 0 || i >= b->count) return fail(QLA_EINVAL, "instance index out of range");
  const int r = b->fit ? fitted_rows(b->ctx[i]->ny, b->rows, b->prefetch, b->fused) : b->rows;
  // the height the kernel realises: whole loop trips of the register window
  const int win = b->prefetch + 4 * b->fused + 2, halo = 4 * b->fused;
  *rows = ((r + 2 * halo + win - 1) / win) * win - 2 * halo;
  return QLA_OK;
}

qla_status qla_batch_destroy(qla_batch* b) {
  if (!b) return QLA_OK;
  DeviceGuard g(b->device);  // frees what it can even if selecting the device fails
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  release_plan(b);
  for (qla_ctx* c : b->ctx) {
    if (!c) continue;
    c->owned_by_batch = false;
    qla_destroy(c);
  }
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return QLA_OK;
}

}  // extern "C"
