// Per-level records and per-kernel-family HIP event timers.
#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.h"

namespace byo {

namespace {
std::mutex g_mu;
bool g_trace_on = false;
bool g_ktimer_on = false;
uint32_t g_ktimer_mask = 0xFFFFFFFFu;  // families that record while timing is on
std::vector<byo_level_record> g_records;
std::vector<hipEvent_t> g_pool;
struct pending_t {
  int family;
  hipEvent_t a, b;
};
std::vector<pending_t> g_pending;
int64_t g_launches[BYO_K_COUNT] = {0};
double g_ms[BYO_K_COUNT] = {0};
}  // namespace

bool trace_on() { return g_trace_on && !noalloc_active(); }
bool ktimer_on() { return g_ktimer_on && !noalloc_active(); }

hipEvent_t event_get() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void event_put(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_pool.push_back(e);
}

void trace_push(const byo_level_record &r) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_records.push_back(r);
}

ktimer_scope::ktimer_scope(int fam, hipStream_t st) : family(fam), s(st) {
  if (!ktimer_on() || !((g_ktimer_mask >> fam) & 1u)) return;
  a = event_get();
  if (a) (void)hipEventRecord(a, s);
}

ktimer_scope::~ktimer_scope() {
  if (!a) return;
  b = event_get();
  if (!b) {
    event_put(a);
    return;
  }
  (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending.push_back({family, a, b});
}

static void drain_locked() {
  for (auto &p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_launches[p.family] += 1;
      g_ms[p.family] += ms;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
}

}  // namespace byo

using namespace byo;

extern "C" {

byo_status byo_trace_enable(int32_t on) {
  g_trace_on = on != 0;
  return BYO_OK;
}

byo_status byo_trace_pending(int64_t *count) {
  BYO_CHECK(count, BYO_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g_mu);
  *count = (int64_t)g_records.size();
  return BYO_OK;
}

byo_status byo_trace_read(byo_level_record *out, int64_t cap, int64_t *count) {
  BYO_CHECK(count && (cap == 0 || out), BYO_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g_mu);
  int64_t k = std::min<int64_t>(cap, (int64_t)g_records.size());
  for (int64_t i = 0; i < k; ++i) out[i] = g_records[i];
  g_records.erase(g_records.begin(), g_records.begin() + k);
  *count = k;
  return BYO_OK;
}

byo_status byo_ktimer_enable(int32_t on) {
  g_ktimer_on = on != 0;
  return BYO_OK;
}

byo_status byo_ktimer_select(uint32_t mask) {
  g_ktimer_mask = mask;
  return BYO_OK;
}

byo_status byo_ktimer_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  for (int i = 0; i < BYO_K_COUNT; ++i) {
    g_launches[i] = 0;
    g_ms[i] = 0;
  }
  return BYO_OK;
}

byo_status byo_ktimer_read(int32_t family, int64_t *launches, double *total_ms) {
  BYO_CHECK(family >= 0 && family < BYO_K_COUNT, BYO_EINVAL, "unknown kernel family");
  BYO_CHECK(launches && total_ms, BYO_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  *launches = g_launches[family];
  *total_ms = g_ms[family];
  return BYO_OK;
}

}  // extern "C"
