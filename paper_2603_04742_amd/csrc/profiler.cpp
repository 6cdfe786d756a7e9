// Per-kernel timing with HIP events recorded around each launch on the launch stream.  Off by
// default; when on, every launcher brackets its kernel with two events and the totals are
// aggregated by kernel name on request.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace hs {

namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_free;

hipEvent_t take_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e;
  HS_CHECK_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

// Launches recorded into a graph are not timed (their events would become graph nodes).
static thread_local bool t_capturing = false;
void profile_capturing(bool on) { t_capturing = on; }

ProfScope::ProfScope(const char* name, hipStream_t st) : name_(name), st_(st) {
  if (t_capturing) return;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_on) return;
  a_ = take_event();
  HS_CHECK_HIP(hipEventRecord(a_, st_));
  active_ = true;
}

ProfScope::~ProfScope() {
  if (!active_) return;
  std::lock_guard<std::mutex> g(g_mu);
  hipEvent_t b = take_event();
  if (hipEventRecord(b, st_) == hipSuccess) g_recs.push_back(Rec{name_, a_, b});
}

void profile_enable(bool on) {
  std::lock_guard<std::mutex> g(g_mu);
  for (Rec& r : g_recs) {
    g_free.push_back(r.a);
    g_free.push_back(r.b);
  }
  g_recs.clear();
  g_on = on;
}

std::string profile_summary() {
  std::lock_guard<std::mutex> g(g_mu);
  std::map<std::string, std::pair<long, double>> agg;
  for (Rec& r : g_recs) {
    HS_CHECK_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    HS_CHECK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    auto& v = agg[r.name];
    v.first++;
    v.second += ms;
  }
  std::string out;
  for (auto& kv : agg) out += kv.first + " " + std::to_string(kv.second.first) + " " + std::to_string(kv.second.second) + "\n";
  return out;
}

}  // namespace hs
