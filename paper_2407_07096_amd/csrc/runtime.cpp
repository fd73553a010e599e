// Host runtime: last-error storage, stream-ordered workspace, small
// host-only entry points of the C ABI.
#include "runtime.h"

#include <cstring>

#include <atomic>
#include <cmath>
#include <map>
#include <mutex>

namespace stag {

namespace {
thread_local std::string g_last_error;
}

stag_status fail(stag_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

void clear_error() { g_last_error.clear(); }

stag_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(STAG_E_DEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
  return STAG_OK;
}

Workspace::~Workspace() {
  for (void* p : ptrs_) (void)hipFreeAsync(p, stream_);
}

namespace {
std::mutex g_pool_mu;
bool g_pool_done[64] = {};
}  // namespace

void keep_pool_memory() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool_done[dev]) return;
  g_pool_done[dev] = true;
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
}

namespace {
std::mutex g_cache_mu;
std::map<int, std::multimap<size_t, void*>> g_cache;
}  // namespace

stag_status cached_alloc(void** p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto& c = g_cache[dev];
    auto it = c.lower_bound(bytes);
    if (it != c.end() && it->first <= 2 * bytes) {
      *p = it->second;
      c.erase(it);
      return STAG_OK;
    }
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? STAG_E_NOMEM : STAG_E_DEVICE, "device allocation of %zu bytes: %s", bytes,
                hipGetErrorString(e));
  }
  return STAG_OK;
}

void cached_free(void* p, size_t bytes) {
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache[dev].emplace(bytes, p);
}

stag_status Workspace::raw_alloc(void** p, size_t bytes) {
  *p = nullptr;
  keep_pool_memory();
  hipError_t e = hipMallocAsync(p, bytes, stream_);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? STAG_E_NOMEM : STAG_E_DEVICE, "workspace allocation of %zu bytes: %s",
                bytes, hipGetErrorString(e));
  }
  ptrs_.push_back(*p);
  return STAG_OK;
}

stag_status Workspace::alloc_bytes(void** p, size_t bytes) {
  *p = nullptr;
  bytes = (bytes + 255) / 256 * 256;
  if (bytes == 0) bytes = 256;
  if (mode_ == kCount) {
    used_ += bytes;
    return STAG_OK;
  }
  if (mode_ == kArena) {
    if (used_ + bytes > cap_)
      return fail(STAG_E_NOMEM, "scratch arena exhausted: %zu + %zu bytes > %zu", used_, bytes, cap_);
    *p = cur_ + used_;
    used_ += bytes;
    return STAG_OK;
  }
  if (bytes >= kSmallBytes) return raw_alloc(p, bytes);
  if (cur_ == nullptr || used_ + bytes > cap_) {
    void* blk = nullptr;
    STAG_TRY(raw_alloc(&blk, kBlockBytes));
    cur_ = static_cast<char*>(blk);
    used_ = 0;
    cap_ = kBlockBytes;
  }
  *p = cur_ + used_;
  used_ += bytes;
  return STAG_OK;
}

namespace {
struct TimerRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_timer_mu;
std::vector<TimerRec> g_timer_recs;
std::atomic<int> g_timing{0};
}  // namespace

bool timing_enabled() { return g_timing.load(std::memory_order_relaxed) != 0; }

ScopedTimer::ScopedTimer(const char* name, hipStream_t s) : name_(name), stream_(s) {
  if (!timing_enabled()) return;
  if (hipEventCreate(&start_) != hipSuccess || hipEventRecord(start_, stream_) != hipSuccess) {
    if (start_) (void)hipEventDestroy(start_);
    start_ = nullptr;
    (void)hipGetLastError();
  }
}

ScopedTimer::~ScopedTimer() {
  if (!start_) return;
  hipEvent_t end = nullptr;
  if (hipEventCreate(&end) != hipSuccess || hipEventRecord(end, stream_) != hipSuccess) {
    if (end) (void)hipEventDestroy(end);
    (void)hipEventDestroy(start_);
    (void)hipGetLastError();
    return;
  }
  std::lock_guard<std::mutex> lk(g_timer_mu);
  g_timer_recs.push_back({name_, start_, end});
}

}  // namespace stag

extern "C" {

void stag_timing_enable(int32_t on) { stag::g_timing.store(on ? 1 : 0); }

// Waits for every recorded launch, then writes "name count total_ms\n" lines
// (one per kernel name, sorted) into buf and clears the records.  Returns
// the number of bytes the full report needs (excluding the terminator).
size_t stag_timing_report(char* buf, size_t len) {
  std::vector<stag::TimerRec> recs;
  {
    std::lock_guard<std::mutex> lk(stag::g_timer_mu);
    recs.swap(stag::g_timer_recs);
  }
  std::map<std::string, std::pair<long, double>> agg;
  for (auto& r : recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& e = agg[r.name];
      e.first += 1;
      e.second += ms;
    }
    (void)hipGetLastError();
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  std::string out;
  char line[256];
  for (auto& kv : agg) {
    snprintf(line, sizeof(line), "%s %ld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  if (buf && len > 0) {
    size_t k = out.size() < len - 1 ? out.size() : len - 1;
    memcpy(buf, out.data(), k);
    buf[k] = 0;
  }
  return out.size();
}

const char* stag_last_error(void) { return stag::g_last_error.c_str(); }

const char* stag_version(void) { return "0.1.0 gfx950"; }

// Closed form of the single-function collision probability (Sec. "Random
// Projection"), written without the overflowing factor exp(8/c^2), boosted
// over K concatenated functions and L tables (Sec. "Boosting the
// Probability").
double stag_e2lsh_collision_probability(double c, int32_t K, int32_t L) {
  if (!(c >= 0.0) || K < 1 || L < 1) return NAN;
  double p = 1.0;
  if (c > 0.0) {
    const double inv_sqrt_2pi = 0.39894228040143267794;  // 1/sqrt(2 pi)
    p = std::erf(2.0 * std::sqrt(2.0) / c) - 0.5 * inv_sqrt_2pi * c * (-std::expm1(-8.0 / (c * c)));
  }
  const double pk = std::pow(p, (double)K);
  if (pk >= 1.0) return 1.0;
  return -std::expm1((double)L * std::log1p(-pk));
}

}  // extern "C"
