// Per-kernel timing with HIP events, for measurement only.  Disabled by
// default; the factorisation itself never depends on it.
#include <mutex>
#include <vector>

#include "../../include/qb.h"
#include "qb_internal.hpp"

namespace qb {
namespace {

struct Pending {
  hipEvent_t start, stop;
  int id;
  double flops, bytes;
};
struct Stat {
  double ms = 0.0, flops = 0.0, bytes = 0.0;
  int64_t launches = 0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
Stat g_stats[kKCount];

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// fold completed pairs into the statistics (caller holds the lock)
int collect_locked() {
  int rc = kOk;
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (p.start && p.stop && hipEventSynchronize(p.stop) == hipSuccess &&
        hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      Stat& s = g_stats[p.id];
      s.ms += ms;
      s.flops += p.flops;
      s.bytes += p.bytes;
      s.launches += 1;
    } else {
      rc = kEHip;
    }
    if (p.start) g_pool.push_back(p.start);
    if (p.stop) g_pool.push_back(p.stop);
  }
  g_pending.clear();
  return rc;
}

const char* kNames[kKCount] = {"sketch", "gemm_nn", "gemm_tn", "reduce", "downdate",
                               "chol_drop", "trinv", "norm", "copy", "gemm_nn_lowp",
                               "gemm_tn_lowp", "gemm_nn_64", "gemm_tn_64", "gemm_nn_256",
                               "batch_sample", "batch_gram", "batch_apply", "batch_reproj",
                               "batch_b", "batch_downdate", "chol_batched", "batch_misc",
                               "sample_i8"};

}  // namespace

const char* kernel_name(int id) { return (id >= 0 && id < kKCount) ? kNames[id] : "unknown"; }

bool prof_enabled() { return g_on; }

int prof_begin(int id, double flops, double bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return -1;
  Pending p{take_event(), take_event(), id, flops, bytes};
  if (p.start) hipEventRecord(p.start, s);
  g_pending.push_back(p);
  return static_cast<int>(g_pending.size()) - 1;
}

void prof_end(int token, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (token < 0 || token >= static_cast<int>(g_pending.size())) return;
  if (g_pending[token].stop) hipEventRecord(g_pending[token].stop, s);
}

}  // namespace qb

using namespace qb;

extern "C" {

int qb_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  collect_locked();
  for (auto& s : g_stats) s = Stat{};
  g_on = (on != 0);
  return QB_OK;
}

int32_t qb_profile_count(void) { return kKCount; }

const char* qb_profile_name(int32_t kernel) { return kernel_name(kernel); }

int qb_profile_read(int32_t kernel, double* ms, int64_t* launches, double* flops, double* bytes) {
  if (kernel < 0 || kernel >= kKCount) return QB_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  const int rc = collect_locked();
  const Stat& s = g_stats[kernel];
  if (ms) *ms = s.ms;
  if (launches) *launches = s.launches;
  if (flops) *flops = s.flops;
  if (bytes) *bytes = s.bytes;
  return rc == kOk ? QB_OK : QB_EHIP;
}

}  // extern "C"
