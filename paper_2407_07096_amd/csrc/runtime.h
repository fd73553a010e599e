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

// Temporary device memory, allocated and released in stream order.
class Workspace {
 public:
  explicit Workspace(hipStream_t s) : stream_(s) {}
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
  stag_status alloc_bytes(void** p, size_t bytes);
  // Hands the allocations to the caller (they are no longer freed here).
  std::vector<void*> release() {
    std::vector<void*> v;
    v.swap(ptrs_);
    return v;
  }

 private:
  hipStream_t stream_;
  std::vector<void*> ptrs_;
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
