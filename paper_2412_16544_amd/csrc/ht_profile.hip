// Optional per-kernel timing with HIP events (include/ht_rise_profile.h).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "ht_internal.h"
#include "ht_rise_profile.h"

namespace ht {

bool g_prof_on = false;

namespace {
struct Rec {
  hipEvent_t a, b;
  int kind;
  double flops, bytes;
};
struct Totals {
  int64_t launches = 0;
  double ms = 0, flops = 0, bytes = 0;
};
std::mutex g_mu;
std::vector<Rec> g_pending;
std::vector<int> g_open;  // indices into g_pending awaiting their end event
std::vector<hipEvent_t> g_pool;
Totals g_tot[(int)KKind::Count];

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void resolve_locked() {
  for (const Rec& r : g_pending) {
    float ms = 0.f;
    if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      Totals& t = g_tot[r.kind];
      t.launches += 1;
      t.ms += ms;
      t.flops += r.flops;
      t.bytes += r.bytes;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_pending.clear();
  g_open.clear();
}
}  // namespace

void prof_begin(KKind k, hipStream_t s, double flops, double bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r{get_event(), get_event(), (int)k, flops, bytes};
  (void)hipEventRecord(r.a, s);
  g_open.push_back((int)g_pending.size());
  g_pending.push_back(r);
}

void prof_end(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_open.empty()) return;
  const int i = g_open.back();
  g_open.pop_back();
  (void)hipEventRecord(g_pending[i].b, s);
  if (g_pending.size() > 4096 && g_open.empty()) resolve_locked();
}

}  // namespace ht

extern "C" {

ht_status ht_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(ht::g_mu);
  ht::resolve_locked();
  for (auto& t : ht::g_tot) t = ht::Totals();
  ht::g_prof_on = on != 0;
  return HT_OK;
}

ht_status ht_profile_read(int32_t kind, ht_kernel_stats* out) {
  if (out == nullptr || kind < 0 || kind >= (int)ht::KKind::Count) return HT_EINVAL;
  std::lock_guard<std::mutex> lk(ht::g_mu);
  ht::resolve_locked();
  const ht::Totals& t = ht::g_tot[kind];
  out->launches = t.launches;
  out->ms = t.ms;
  out->flops = t.flops;
  out->bytes = t.bytes;
  return HT_OK;
}

int32_t ht_profile_kind_count(void) { return (int32_t)ht::KKind::Count; }

const char* ht_profile_kind_name(int32_t kind) {
  static const char* names[] = {"sumsq",        "gram",         "ttm_contract",         "ttm_expand",
                                "eig_trunc",    "orth_expand",  "layout",               "gram_f32",
                                "ttm_contract_f32", "gram_f32_reg", "ttm_contract_f32_reg", "gram_reg64",
                                "ttm_contract_reg64"};
  if (kind < 0 || kind >= (int)ht::KKind::Count) return "";
  return names[kind];
}

}  // extern "C"
