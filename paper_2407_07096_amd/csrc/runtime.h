// Host runtime shared by the library's entry points: status/last-error
// handling, stream-ordered workspace, launch checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/stag_kde.h"

namespace stag {

// Records a message for stag_last_error() and returns the status.
stag_status fail(stag_status st, const char* fmt, ...);
void clear_error();

#define STAG_HIP(expr)                                                                        \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return ::stag::fail(STAG_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                          __FILE__, __LINE__);                                                \
  } while (0)

#define STAG_TRY(expr)                  \
  do {                                  \
    stag_status s_ = (expr);            \
    if (s_ != STAG_OK) return s_;       \
  } while (0)

// Checks the launch that was just issued.
stag_status check_launch(const char* what);

// Sets `bytes` bytes at device pointer p to zero with a fill kernel on stream
// st (in stream order; used instead of a memset where the call may be recorded
// into a HIP graph).
stag_status zero_async(void* p, size_t bytes, hipStream_t st);

// Temporary device memory, allocated and released in stream order.
// The current device's default stream-ordered pool keeps freed memory for
// reuse (release threshold at the maximum) instead of returning it to the
// system at every synchronisation; set once per device on first use.
void keep_pool_memory();

// Long-lived device blocks (index memory) with a per-device cache: a freed
// block is kept and handed to a later request of at most its size (and at
// least half of it) on the same device; blocks are returned to the system
// only at process exit.  cached_free requires the block to be idle.
stag_status cached_alloc(void** p, size_t bytes);
void cached_free(void* p, size_t bytes);

class Workspace {
 public:
  explicit Workspace(hipStream_t s) : stream_(s) {}
  // Arena: every request is a 256-byte-aligned slice of the caller's
  // device buffer [base, base + cap); nothing is allocated or freed, and a
  // request past the end fails.
  Workspace(hipStream_t s, void* base, size_t cap)
      : stream_(s), mode_(kArena), cur_(static_cast<char*>(base)), cap_(cap) {}
  // Counter: requests only add up their (aligned) sizes, read by used(); the
  // pointers handed out are null and must not reach a launch.
  struct CountTag {};
  explicit Workspace(CountTag) : stream_(nullptr), mode_(kCount) {}
  size_t used() const { return used_; }
  ~Workspace();
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  template <typename T>
  stag_status alloc(T** p, size_t count) {
    void* v = nullptr;
    stag_status st = alloc_bytes(&v, count * sizeof(T));
    *p = static_cast<T*>(v);
    return st;
  }
  // Requests below kSmallBytes share kBlockBytes blocks (256-byte aligned
  // slices); larger ones get an allocation of their own.  Every pool
  // allocation and stream-ordered free costs host time on the caller's
  // critical path, so the blocks are large: a call's temporaries (sort
  // buffers, scans, partial sums of up to 32 MiB each) then come from one or
  // two pool allocations.
  stag_status alloc_bytes(void** p, size_t bytes);
  // Hands the allocations to the caller (they are no longer freed here).
  std::vector<void*> release() {
    std::vector<void*> v;
    v.swap(ptrs_);
    cur_ = nullptr;
    used_ = cap_ = 0;
    return v;
  }
  static constexpr size_t kSmallBytes = (size_t)32 << 20;
  static constexpr size_t kBlockBytes = (size_t)64 << 20;

 private:
  stag_status raw_alloc(void** p, size_t bytes);
  enum Mode { kPool, kArena, kCount };
  hipStream_t stream_;
  Mode mode_ = kPool;
  std::vector<void*> ptrs_;
  char* cur_ = nullptr;
  size_t used_ = 0, cap_ = 0;
};

// Optional per-kernel timing: when enabled, ScopedTimer records a HIP event
// pair around a launch on its stream; stag_timing_report() aggregates them.
bool timing_enabled();
class ScopedTimer {
 public:
  ScopedTimer(const char* name, hipStream_t s);
  ~ScopedTimer();
  ScopedTimer(const ScopedTimer&) = delete;
  ScopedTimer& operator=(const ScopedTimer&) = delete;

 private:
  const char* name_;
  hipStream_t stream_;
  hipEvent_t start_ = nullptr;
};

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }

}  // namespace stag
