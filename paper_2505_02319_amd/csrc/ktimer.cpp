#include "ktimer.h"

#include <mutex>
#include <vector>

#include "common.h"

namespace ikr {

namespace {

struct Pending {
  int id;
  hipEvent_t a, b;
  double bytes;
};

struct State {
  std::mutex mu;
  unsigned mask = 0;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t open[K_COUNT] = {};
  long long launches[K_COUNT] = {};
  double ms[K_COUNT] = {};
  double bytes[K_COUNT] = {};
};

State& S() {
  static State s;
  return s;
}

hipEvent_t get_event(State& s) {
  if (!s.pool.empty()) {
    hipEvent_t e = s.pool.back();
    s.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  IKR_HIP(hipEventCreate(&e));
  return e;
}

void resolve(State& s) {
  for (Pending& p : s.pending) {
    IKR_HIP(hipEventSynchronize(p.b));
    float t = 0;
    IKR_HIP(hipEventElapsedTime(&t, p.a, p.b));
    s.launches[p.id] += 1;
    s.ms[p.id] += t;
    s.bytes[p.id] += p.bytes;
    s.pool.push_back(p.a);
    s.pool.push_back(p.b);
  }
  s.pending.clear();
}

}  // namespace

const char* kernel_name(int id) {
  static const char* names[K_COUNT] = {
      "col_inv", "plane_hv", "col_fwd", "gram", "update", "cg_step", "plane_rho",
      "col_inv_fp32", "plane_hv_fp32", "col_fwd_fp32", "gram_fp32", "update_fp32",
      "cg_step_fp32"};
  return (id >= 0 && id < K_COUNT) ? names[id] : "?";
}

void KTimer::enable(unsigned mask) {
  std::lock_guard<std::mutex> g(S().mu);
  S().mask = mask;
}

bool KTimer::enabled() { return S().mask != 0; }

void KTimer::begin(int id, hipStream_t st) {
  State& s = S();
  if (!((s.mask >> id) & 1u)) return;
  std::lock_guard<std::mutex> g(s.mu);
  hipEvent_t e = get_event(s);
  IKR_HIP(hipEventRecord(e, st));
  s.open[id] = e;
}

void KTimer::end(int id, hipStream_t st, double bytes) {
  State& s = S();
  if (!((s.mask >> id) & 1u)) return;
  std::lock_guard<std::mutex> g(s.mu);
  if (!s.open[id]) return;
  hipEvent_t e = get_event(s);
  IKR_HIP(hipEventRecord(e, st));
  s.pending.push_back(Pending{id, s.open[id], e, bytes});
  s.open[id] = nullptr;
  if (s.pending.size() > 4096) resolve(s);
}

void KTimer::add_bytes(int id, double bytes) {
  State& s = S();
  if (id < 0 || id >= K_COUNT || !((s.mask >> id) & 1u)) return;
  std::lock_guard<std::mutex> g(s.mu);
  s.bytes[id] += bytes;
}

void KTimer::query(int id, long long* launches, double* ms, double* bytes) {
  State& s = S();
  std::lock_guard<std::mutex> g(s.mu);
  resolve(s);
  if (launches) *launches = s.launches[id];
  if (ms) *ms = s.ms[id];
  if (bytes) *bytes = s.bytes[id];
}

void KTimer::reset() {
  State& s = S();
  std::lock_guard<std::mutex> g(s.mu);
  resolve(s);
  for (int i = 0; i < K_COUNT; ++i) {
    s.launches[i] = 0;
    s.ms[i] = 0;
    s.bytes[i] = 0;
  }
}

}  // namespace ikr
