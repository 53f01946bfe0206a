// Optional per-kernel timing with HIP events recorded on the launch stream.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace mialign {
namespace {

struct Pending {
  std::string name;
  hipEvent_t start, stop;
};

struct ProfState {
  std::mutex mu;
  bool enabled = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<int64_t, double>> acc;
};

ProfState& state() {
  static ProfState* st = new ProfState();  // never destroyed: events may outlive static teardown order
  return *st;
}

hipEvent_t take_event(ProfState& st) {
  if (!st.pool.empty()) {
    hipEvent_t e = st.pool.back();
    st.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain(ProfState& st) {
  for (auto& p : st.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      auto& a = st.acc[p.name];
      a.first += 1;
      a.second += ms;
    }
    st.pool.push_back(p.start);
    st.pool.push_back(p.stop);
  }
  st.pending.clear();
}

}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t stream) : token_(-1), stream_(stream) {
  ProfState& st = state();
  std::lock_guard<std::mutex> g(st.mu);
  if (!st.enabled) return;
  Pending p;
  p.name = name;
  p.start = take_event(st);
  p.stop = take_event(st);
  if (!p.start || !p.stop) return;
  hipEventRecord(p.start, stream);
  st.pending.push_back(p);
  token_ = (int)st.pending.size() - 1;
}

ProfScope::~ProfScope() {
  if (token_ < 0) return;
  ProfState& st = state();
  std::lock_guard<std::mutex> g(st.mu);
  if (token_ < (int)st.pending.size()) hipEventRecord(st.pending[token_].stop, stream_);
}

}  // namespace mialign

using namespace mialign;

extern "C" {

aln_status_t aln_profile_enable(int on) {
  ProfState& st = state();
  std::lock_guard<std::mutex> g(st.mu);
  st.enabled = on != 0;
  return ALN_OK;
}

aln_status_t aln_profile_reset(void) {
  ProfState& st = state();
  std::lock_guard<std::mutex> g(st.mu);
  drain(st);
  st.acc.clear();
  return ALN_OK;
}

aln_status_t aln_profile_read(aln_profile_entry_t* entries, int32_t max_entries, int32_t* n_entries) {
  if (!n_entries || (max_entries > 0 && !entries)) return ALN_E_INVALID;
  ProfState& st = state();
  std::lock_guard<std::mutex> g(st.mu);
  drain(st);
  int32_t k = 0;
  for (auto& kv : st.acc) {
    if (k < max_entries) {
      std::memset(entries[k].name, 0, sizeof(entries[k].name));
      std::strncpy(entries[k].name, kv.first.c_str(), sizeof(entries[k].name) - 1);
      entries[k].launches = kv.second.first;
      entries[k].total_ms = kv.second.second;
    }
    ++k;
  }
  *n_entries = k;
  return ALN_OK;
}

}  // extern "C"
