#include "profile.hpp"

#include <map>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace spaqr {

namespace {
struct Rec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  int64_t launches = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
};
std::mutex g_mu;
bool g_on = false;
std::string g_only;  // record only this kernel when non-empty
std::map<std::string, Rec> g_tab;

void resolve(Rec& r) {
  for (auto& e : r.ev) {
    float t = 0.f;
    (void)hipEventSynchronize(e.second);
    if (hipEventElapsedTime(&t, e.first, e.second) == hipSuccess) r.ms += t;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  r.ev.clear();
}
}  // namespace

bool prof_on() { return g_on; }
// `only` names one timer, or with a trailing '*' every timer of that prefix
bool prof_wants(const char* name) {
  if (!g_on) return false;
  if (g_only.empty()) return true;
  if (g_only.back() == '*') return std::strncmp(name, g_only.c_str(), g_only.size() - 1) == 0;
  return g_only == name;
}

void prof_record(const char* name, hipStream_t, hipEvent_t a, hipEvent_t b, double flops, double bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  Rec& r = g_tab[name];
  r.ev.emplace_back(a, b);
  r.launches++;
  r.flops += flops;
  r.bytes += bytes;
  if (r.ev.size() > 4096) resolve(r);
}

void prof_host(const char* name, double ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  Rec& r = g_tab[name];
  r.launches++;
  r.ms += ms;
}

namespace {
std::mutex g_cmu;
std::map<std::string, int64_t> g_count;
}  // namespace

void count_launch(const char* kernel) {
  std::lock_guard<std::mutex> lk(g_cmu);
  ++g_count[kernel];
}

void prof_add(const char* name, double flops, double bytes) {
  if (!prof_wants(name)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec& r = g_tab[name];
  r.flops += flops;
  r.bytes += bytes;
}

}  // namespace spaqr

extern "C" {

spaqr_status spaqr_profile_enable(int on, const char* only) {
  std::lock_guard<std::mutex> lk(spaqr::g_mu);
  for (auto& kv : spaqr::g_tab) spaqr::resolve(kv.second);
  spaqr::g_tab.clear();
  spaqr::g_on = on != 0;
  spaqr::g_only = only ? only : "";
  return SPAQR_OK;
}

spaqr_status spaqr_kernel_launches(const char* kernel, int64_t* count) {
  if (!count) return SPAQR_EINVAL;
  std::lock_guard<std::mutex> lk(spaqr::g_cmu);
  if (!kernel) {
    spaqr::g_count.clear();
    *count = 0;
    return SPAQR_OK;
  }
  auto it = spaqr::g_count.find(kernel);
  *count = it == spaqr::g_count.end() ? 0 : it->second;
  return SPAQR_OK;
}

void spaqr_prof_release() {
  std::lock_guard<std::mutex> lk(spaqr::g_mu);
  for (auto& kv : spaqr::g_tab) spaqr::resolve(kv.second);
  spaqr::g_tab.clear();
  spaqr::g_on = false;
  spaqr::g_only.clear();
}

spaqr_status spaqr_profile_query(const char* name, int64_t* launches, double* total_ms, double* flops,
                                 double* bytes) {
  if (!name) return SPAQR_EINVAL;
  std::lock_guard<std::mutex> lk(spaqr::g_mu);
  auto it = spaqr::g_tab.find(name);
  if (it == spaqr::g_tab.end()) {
    if (launches) *launches = 0;
    if (total_ms) *total_ms = 0.0;
    if (flops) *flops = 0.0;
    if (bytes) *bytes = 0.0;
    return SPAQR_OK;
  }
  spaqr::resolve(it->second);
  if (launches) *launches = it->second.launches;
  if (total_ms) *total_ms = it->second.ms;
  if (flops) *flops = it->second.flops;
  if (bytes) *bytes = it->second.bytes;
  return SPAQR_OK;
}

}  // extern "C"
