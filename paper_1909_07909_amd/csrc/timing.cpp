#include "timing.hpp"

#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hss.h"

namespace hss {
namespace {
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex mu;
bool enabled = false;
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;
Rec* open_rec = nullptr;

hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  (void)hipEventCreate(&e);
  return e;
}
}  // namespace

bool timing_on() { return enabled; }

void timing_begin(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> g(mu);
  recs.push_back(Rec{name, get_event(), get_event()});
  (void)hipEventRecord(recs.back().a, s);
}

void timing_end(hipStream_t s) {
  std::lock_guard<std::mutex> g(mu);
  if (!recs.empty()) (void)hipEventRecord(recs.back().b, s);
}

}  // namespace hss

using namespace hss;

extern "C" {

hss_status hss_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> g(mu);
  enabled = on != 0;
  return HSS_OK;
}

hss_status hss_timing_report(char* buf, int64_t cap, int32_t reset) {
  if (!buf && cap > 0) return -1;
  std::lock_guard<std::mutex> g(mu);
  std::map<std::string, std::pair<double, long>> agg;
  for (Rec& r : recs) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0.f;
    auto& x = agg[r.name];
    x.first += ms;
    x.second += 1;
  }
  std::string out = "[";
  bool first = true;
  for (auto& kv : agg) {
    char line[256];
    std::snprintf(line, sizeof line, "%s{\"kernel\": \"%s\", \"launches\": %ld, \"total_ms\": %.6f}",
                  first ? "" : ", ", kv.first.c_str(), kv.second.second, kv.second.first);
    out += line;
    first = false;
  }
  out += "]";
  if (reset) {
    for (Rec& r : recs) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  if (cap > 0) {
    std::snprintf(buf, (size_t)cap, "%s", out.c_str());
  }
  return (int64_t)out.size() + 1 > cap ? HSS_EUNSUP : HSS_OK;
}

}  // extern "C"
