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
  long units;
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
// Units of work (key switches of a rotation level) of the launches the calling thread makes next.
static thread_local long t_units = 0;
ProfUnits::ProfUnits(long n) : prev_(t_units) { t_units = n; }
ProfUnits::~ProfUnits() { t_units = prev_; }

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
  if (hipEventRecord(b, st_) == hipSuccess) g_recs.push_back(Rec{name_, a_, b, t_units});
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
  struct Agg {
    long n = 0, units = 0;
    double ms = 0;
  };
  std::map<std::string, Agg> agg;
  for (Rec& r : g_recs) {
    HS_CHECK_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    HS_CHECK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    Agg& v = agg[r.name];
    v.n++;
    v.ms += ms;
    v.units += r.units;
  }
  std::string out;
  for (auto& kv : agg)
    out += kv.first + " " + std::to_string(kv.second.n) + " " + std::to_string(kv.second.ms) + " " + std::to_string(kv.second.units) + "\n";
  return out;
}

}  // namespace hs
