// Continuous-batching request scheduler for kernel-density queries against
// resident data sets (host C++, no device code).  The device side is behind
// the Executor interface so the same scheduler drives the GPU executor of the
// library and a mock executor in the host-only tests.
//
// Policy:
//   arrival  FIFO queue; submit() is thread safe.
//   admit    the head request is admitted when its workspace footprint fits
//            the remaining budget, otherwise the queue waits (FIFO order); a
//            request larger than the whole budget is rejected at submission
//            (status STAG_E_BUSY).
//   chunk    an admitted request is served in chunks of at most
//            chunk_queries queries (its rows in order), so that a large
//            request does not hold a stream for its whole length.
//   batch    every idle stream takes the oldest admitted request that still
//            has rows to start and packs the next chunk of every admitted
//            request with the same data set and key (arrival order, at most
//            one chunk per request) behind it, up to max_batch_queries
//            queries and the executor's item limit, then launches them as
//            one batch.  Small requests that arrive behind a large one thus
//            share the next batches instead of waiting for all its chunks.
//   retire   a finished stream retires its batch: per-chunk status; a
//            request completes when its last chunk is retired (latency from
//            arrival to that moment) and its footprint is released.
// A failure reported for one chunk fails only its request.
#pragma once

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace stag {
namespace serve {

struct Request {
  uint64_t id = 0;
  int dataset = 0;
  int key = 0;  // batching key: requests of one batch share data set and key
  int64_t m = 0;
  const void* Q = nullptr;
  void* S = nullptr;
  void* B = nullptr;  // optional second output (per-result bounds)
  size_t footprint = 0;
  double t_submit = 0.0, t_admit = 0.0, t_launch = 0.0, t_done = 0.0;
  int64_t next_row = 0;  // first row not yet in a launched chunk
  int outstanding = 0;   // launched chunks not yet retired
  int status = -1;       // -1 pending, else a stag_status
  bool done = false;
};

// One chunk of a request: rows [row0, row0 + m).
struct Item {
  Request* r = nullptr;
  int64_t row0 = 0, m = 0;
};

class Executor {
 public:
  virtual ~Executor() = default;
  virtual int n_streams() const = 0;
  virtual double now() = 0;
  // Largest number of items one batch may hold.
  virtual int max_batch_items() const = 0;
  // Workspace bytes a request of m queries with this key on data set ds
  // needs (0: invalid).
  virtual size_t footprint(int ds, int key, int64_t m) = 0;
  // Starts a batch on `stream` (asynchronously).  Returns a stag_status; on
  // failure nothing is running on the stream.
  virtual int launch(int ds, int key, const std::vector<Item>& batch, int stream) = 0;
  // True once the batch last launched on `stream` has finished.
  virtual bool finished(int stream) = 0;
  // Statuses of that batch's items (in batch order); releases resources.
  virtual std::vector<int> retire(int stream) = 0;
};

struct Stats {
  uint64_t submitted = 0, completed = 0, failed = 0, rejected = 0, batches = 0;
  double p50 = 0.0, p99 = 0.0, mean = 0.0, max = 0.0;  // latency in seconds
  uint64_t queries = 0;                                  // completed queries
  size_t inflight_bytes = 0, peak_inflight_bytes = 0;
};

class Scheduler {
 public:
  Scheduler(Executor* ex, size_t budget_bytes, int64_t max_batch_queries, int64_t chunk_queries);
  ~Scheduler();

  // Enqueues a request; returns its ticket (> 0), or 0 if it is invalid.
  uint64_t submit(int ds, int key, const void* Q, int64_t m, void* S, void* B = nullptr);
  // One scheduling round: retire finished batches, admit, launch.  Returns
  // true if anything changed.
  bool step();
  // Runs step() on a worker thread until stop() (GPU use).
  void start();
  void stop();
  // Blocks until the ticket is done (worker mode); returns its status.
  int wait(uint64_t ticket, double* latency_s);
  // Non-blocking: 1 done, 0 pending, -1 unknown ticket.
  int poll(uint64_t ticket, int* status, double* latency_s);
  Stats stats();
  bool idle();

 private:
  bool step_locked();
  void finish_locked(Request* r, double t);
  Executor* ex_;
  size_t budget_;
  int64_t max_batch_;
  int64_t chunk_;
  std::mutex mu_;
  std::condition_variable cv_done_, cv_work_;
  std::deque<Request*> queue_;  // submitted, not admitted
  std::deque<Request*> ready_;  // admitted, rows left to start
  std::map<uint64_t, std::unique_ptr<Request>> all_;
  std::vector<std::vector<Item>> running_;
  std::vector<double> latencies_;
  uint64_t next_id_ = 1;
  Stats st_;
  bool stop_ = false;
  std::thread worker_;
};

}  // namespace serve
}  // namespace stag
