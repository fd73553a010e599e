// Host-only test harness for the serving scheduler: a mock executor with a
// virtual clock (batch time = c0 + c1 * queries), a per-query workspace
// footprint, a limit of items per batch and an injectable device failure,
// behind a small C API that the Python tests drive.  Test infrastructure; not part of the library.
#include <cstdint>
#include <vector>

#include "serve_core.h"

namespace {

constexpr uintptr_t kFailTag = 0xBAD00000;

class MockExecutor : public stag::serve::Executor {
 public:
  MockExecutor(int ns, double c0, double c1, size_t bpq, int max_items)
      : ns_(ns), c0_(c0), c1_(c1), bpq_(bpq), max_items_(max_items), busy_until_(ns, -1.0), batches_(ns) {}
  int n_streams() const override { return ns_; }
  double now() override { return t_; }
  int max_batch_items() const override { return max_items_; }
  size_t footprint(int ds, int key, int64_t m) override { return ds < 0 || key < 0 ? 0 : (size_t)m * bpq_; }
  int launch(int ds, int key, const std::vector<stag::serve::Item>& batch, int s) override {
    if (ds == 99) return 3;  // a launch failure for data set 99
    if ((int)batch.size() > max_items_) return 1;  // the scheduler must never do this
    int64_t q = 0;
    for (auto& it : batch) q += it.m;
    busy_until_[s] = t_ + c0_ + c1_ * (double)q;
    batches_[s] = batch;
    log_.push_back({s, ds, (int)batch.size(), q, key});
    return 0;
  }
  bool finished(int s) override { return busy_until_[s] < 0.0 || t_ >= busy_until_[s]; }
  std::vector<int> retire(int s) override {
    std::vector<int> st;
    for (auto& it : batches_[s])
      st.push_back(((uintptr_t)it.r->Q & 0xFFF00000u) == kFailTag ? 3 : 0);
    busy_until_[s] = -1.0;
    batches_[s].clear();
    return st;
  }
  double t_ = 0.0;
  struct Launch {
    int stream, ds, nreq;
    int64_t queries;
    int key;
  };
  std::vector<Launch> log_;

 private:
  int ns_;
  double c0_, c1_;
  size_t bpq_;
  int max_items_;
  std::vector<double> busy_until_;
  std::vector<std::vector<stag::serve::Item>> batches_;
};

struct Mock {
  MockExecutor ex;
  stag::serve::Scheduler sched;
  Mock(size_t budget, int ns, int64_t maxb, double c0, double c1, size_t bpq, int64_t chunk, int max_items)
      : ex(ns, c0, c1, bpq, max_items), sched(&ex, budget, maxb, chunk) {}
};

}  // namespace

extern "C" {

void* mock_create(uint64_t budget, int32_t ns, int64_t maxb, double c0, double c1, uint64_t bpq, int64_t chunk,
                  int32_t max_items) {
  return new Mock(budget, ns, maxb, c0, c1, bpq, chunk, max_items);
}
void mock_destroy(void* h) { delete static_cast<Mock*>(h); }

uint64_t mock_submit(void* h, int32_t ds, int64_t m, int32_t fail, int32_t key) {
  Mock* mk = static_cast<Mock*>(h);
  static uintptr_t counter = 0x1000;
  counter += 16;
  const void* Q = reinterpret_cast<const void*>(fail ? (kFailTag | (counter & 0xFFFFF)) : counter);
  return mk->sched.submit(ds, key, Q, m, reinterpret_cast<void*>(counter));
}

// Runs scheduling rounds at the current virtual time until nothing changes,
// advances the clock by dt, and runs rounds again.
void mock_advance(void* h, double dt) {
  Mock* mk = static_cast<Mock*>(h);
  while (mk->sched.step()) {
  }
  mk->ex.t_ += dt;
  while (mk->sched.step()) {
  }
}

int32_t mock_poll(void* h, uint64_t ticket, int32_t* status, double* latency) {
  int st = 0;
  const int r = static_cast<Mock*>(h)->sched.poll(ticket, &st, latency);
  if (status) *status = st;
  return r;
}

void mock_stats(void* h, double* out) {
  const stag::serve::Stats s = static_cast<Mock*>(h)->sched.stats();
  out[0] = (double)s.submitted;
  out[1] = (double)s.completed;
  out[2] = (double)s.failed;
  out[3] = (double)s.rejected;
  out[4] = (double)s.batches;
  out[5] = (double)s.queries;
  out[6] = s.p50;
  out[7] = s.p99;
  out[8] = s.mean;
  out[9] = s.max;
  out[10] = (double)s.inflight_bytes;
  out[11] = (double)s.peak_inflight_bytes;
}

int32_t mock_launches(void* h, int32_t* out, int32_t cap) {
  auto& lg = static_cast<Mock*>(h)->ex.log_;
  int32_t k = 0;
  for (auto& l : lg) {
    if (k + 5 > cap) break;
    out[k++] = l.stream;
    out[k++] = l.ds;
    out[k++] = l.nreq;
    out[k++] = (int32_t)l.queries;
    out[k++] = l.key;
  }
  return (int32_t)lg.size();
}

}  // extern "C"
