// HIP-event profiler behind fgs_profile_enable / fgs_profile_read.
#include <mutex>
#include <vector>

#include "fgs_internal.hpp"

namespace fgs {
namespace {

const char* const kNames[kKNumKernels] = {
    "preprocess", "compact", "depth_sort_hist", "depth_sort_scatter", "scan", "duplicate", "tile_sort_hist",
    "tile_sort_scatter", "ranges", "fill", "blend_forward", "blend_backward", "preprocess_backward",
    "color", "rows", "loss", "spatial_order",
    "grad_segreduce", "duplicate_hist"};

struct Record {
  int id;
  hipEvent_t start, stop;
};

struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<Record> pending;
  int64_t launches[kKNumKernels] = {};
  double total_ms[kKNumKernels] = {};

  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

Profiler& prof() {
  static Profiler p;
  return p;
}

}  // namespace

const char* kernel_name(int id) { return (id >= 0 && id < kKNumKernels) ? kNames[id] : "?"; }

ProfScope::ProfScope(hipStream_t s, int id) : s_(s), slot_(-1) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  if (!p.on) return;
  Record r{id, p.get_event(), p.get_event()};
  if (!r.start || !r.stop) return;
  if (hipEventRecord(r.start, s) != hipSuccess) return;
  p.pending.push_back(r);
  slot_ = (int)p.pending.size() - 1;
}

ProfScope::~ProfScope() {
  if (slot_ < 0) return;
  Profiler& p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  if (slot_ < (int)p.pending.size()) (void)hipEventRecord(p.pending[slot_].stop, s_);
}

}  // namespace fgs

using namespace fgs;

extern "C" int fgs_profile_enable(int32_t on) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  if (on) {
    for (auto& r : p.pending) {
      (void)hipEventSynchronize(r.stop);
      p.pool.push_back(r.start);
      p.pool.push_back(r.stop);
    }
    p.pending.clear();
    for (int k = 0; k < kKNumKernels; ++k) {
      p.launches[k] = 0;
      p.total_ms[k] = 0.0;
    }
  }
  p.on = on != 0;
  return FGS_OK;
}

extern "C" int fgs_profile_read(fgs_profile* out) {
  if (!out) return FGS_ERR_ARG;
  Profiler& p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  for (auto& r : p.pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      p.launches[r.id] += 1;
      p.total_ms[r.id] += ms;
    }
    p.pool.push_back(r.start);
    p.pool.push_back(r.stop);
  }
  p.pending.clear();
  out->count = kKNumKernels;
  for (int k = 0; k < FGS_PROF_MAX_KERNELS; ++k) {
    out->names[k] = k < kKNumKernels ? kNames[k] : nullptr;
    out->launches[k] = k < kKNumKernels ? p.launches[k] : 0;
    out->total_ms[k] = k < kKNumKernels ? p.total_ms[k] : 0.0;
  }
  return FGS_OK;
}
