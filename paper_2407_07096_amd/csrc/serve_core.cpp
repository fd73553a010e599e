// Continuous-batching scheduler (see serve_core.h).
#include "serve_core.h"

#include <algorithm>
#include <chrono>
#include <cmath>

namespace stag {
namespace serve {

namespace {
constexpr int kOk = 0;
constexpr int kBusy = 5;
constexpr int kInval = 1;

double pct(std::vector<double> v, double p) {  // nearest-rank percentile
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::ceil(p / 100.0 * (double)v.size());
  if (k < 1) k = 1;
  return v[k - 1];
}
}  // namespace

Scheduler::Scheduler(Executor* ex, size_t budget_bytes, int64_t max_batch_queries, int64_t chunk_queries)
    : ex_(ex), budget_(budget_bytes), max_batch_(max_batch_queries), chunk_(chunk_queries > 0 ? chunk_queries : 1) {
  running_.resize((size_t)ex_->n_streams());
}

Scheduler::~Scheduler() { stop(); }

uint64_t Scheduler::submit(int ds, int key, const void* Q, int64_t m, void* S, void* B) {
  if (m < 1 || !Q || !S) return 0;
  std::unique_ptr<Request> r(new Request());
  r->dataset = ds;
  r->key = key;
  r->m = m;
  r->Q = Q;
  r->S = S;
  r->B = B;
  r->footprint = ex_->footprint(ds, key, m);
  if (r->footprint == 0) return 0;
  std::lock_guard<std::mutex> lk(mu_);
  r->id = next_id_++;
  r->t_submit = ex_->now();
  const uint64_t id = r->id;
  st_.submitted++;
  if (r->footprint > budget_) {  // can never be admitted
    r->status = kBusy;
    r->done = true;
    r->t_done = r->t_submit;
    st_.rejected++;
    all_[id] = std::move(r);
    cv_done_.notify_all();
    return id;
  }
  queue_.push_back(r.get());
  all_[id] = std::move(r);
  cv_work_.notify_all();
  return id;
}

bool Scheduler::step() {
  std::lock_guard<std::mutex> lk(mu_);
  return step_locked();
}

void Scheduler::finish_locked(Request* r, double t) {
  r->t_done = t;
  r->done = true;
  st_.inflight_bytes -= r->footprint;
  if (r->status == kOk) {
    st_.completed++;
    st_.queries += (uint64_t)r->m;
    latencies_.push_back(r->t_done - r->t_submit);
  } else {
    st_.failed++;
  }
}

bool Scheduler::step_locked() {
  bool changed = false;
  const int ns = ex_->n_streams();
  // retire
  for (int s = 0; s < ns; ++s) {
    if (running_[s].empty() || !ex_->finished(s)) continue;
    std::vector<int> sts = ex_->retire(s);
    const double t = ex_->now();
    for (size_t k = 0; k < running_[s].size(); ++k) {
      Request* r = running_[s][k].r;
      const int stk = k < sts.size() ? sts[k] : kOk;
      if (r->status == -1 || r->status == kOk) r->status = stk;  // the first failure sticks
      r->outstanding--;
      if (r->outstanding == 0 && r->next_row >= r->m) finish_locked(r, t);
    }
    running_[s].clear();
    changed = true;
  }
  if (changed) cv_done_.notify_all();
  // admit (FIFO; the head blocks while it does not fit)
  while (!queue_.empty()) {
    Request* r = queue_.front();
    if (st_.inflight_bytes + r->footprint > budget_) break;
    queue_.pop_front();
    st_.inflight_bytes += r->footprint;
    st_.peak_inflight_bytes = std::max(st_.peak_inflight_bytes, st_.inflight_bytes);
    r->t_admit = ex_->now();
    r->status = kOk;
    ready_.push_back(r);
    changed = true;
  }
  // launch on idle streams: the oldest request with rows left sets the data
  // set and key; every ready request of that data set and key gives its next
  // chunk, in arrival order, while the batch has room
  const int max_items = std::max(1, ex_->max_batch_items());
  for (int s = 0; s < ns && !ready_.empty(); ++s) {
    if (!running_[s].empty()) continue;
    const int ds = ready_.front()->dataset, key = ready_.front()->key;
    std::vector<Item> batch;
    int64_t q = 0;
    for (auto it = ready_.begin(); it != ready_.end() && (int)batch.size() < max_items;) {
      Request* r = *it;
      if (r->dataset != ds || r->key != key) {
        ++it;
        continue;
      }
      const int64_t take = std::min(chunk_, r->m - r->next_row);
      if (!batch.empty() && q + take > max_batch_) break;
      batch.push_back(Item{r, r->next_row, take});
      q += take;
      r->next_row += take;
      r->outstanding++;
      if (r->next_row >= r->m) it = ready_.erase(it);
      else ++it;
    }
    const double t = ex_->now();
    for (Item& b : batch)
      if (b.row0 == 0) b.r->t_launch = t;
    const int rc = ex_->launch(ds, key, batch, s);
    if (rc != kOk) {
      for (Item& b : batch) {
        Request* r = b.r;
        r->status = rc;
        r->outstanding--;
        if (r->next_row < r->m) {  // its remaining rows are not started
          r->next_row = r->m;
          for (auto it = ready_.begin(); it != ready_.end(); ++it)
            if (*it == r) {
              ready_.erase(it);
              break;
            }
        }
        if (r->outstanding == 0) finish_locked(r, t);
      }
      cv_done_.notify_all();
    } else {
      running_[s] = batch;
      st_.batches++;
    }
    changed = true;
  }
  return changed;
}

void Scheduler::start() {
  std::lock_guard<std::mutex> lk(mu_);
  if (worker_.joinable()) return;
  stop_ = false;
  worker_ = std::thread([this] {
    std::unique_lock<std::mutex> lk2(mu_);
    while (!stop_) {
      const bool changed = step_locked();
      bool busy = false;
      for (auto& b : running_) busy = busy || !b.empty();
      if (!changed) {
        if (busy) {
          lk2.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          lk2.lock();
        } else {
          cv_work_.wait_for(lk2, std::chrono::milliseconds(5));
        }
      }
    }
  });
}

void Scheduler::stop() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
    cv_work_.notify_all();
  }
  if (worker_.joinable()) worker_.join();
}

int Scheduler::wait(uint64_t ticket, double* latency_s) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) return kInval;
  Request* r = it->second.get();
  cv_done_.wait(lk, [&] { return r->done; });
  if (latency_s) *latency_s = r->t_done - r->t_submit;
  return r->status;
}

int Scheduler::poll(uint64_t ticket, int* status, double* latency_s) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) return -1;
  Request* r = it->second.get();
  if (!r->done) return 0;
  if (status) *status = r->status;
  if (latency_s) *latency_s = r->t_done - r->t_submit;
  return 1;
}

Stats Scheduler::stats() {
  std::lock_guard<std::mutex> lk(mu_);
  Stats s = st_;
  s.p50 = pct(latencies_, 50.0);
  s.p99 = pct(latencies_, 99.0);
  double sum = 0.0, mx = 0.0;
  for (double v : latencies_) {
    sum += v;
    mx = std::max(mx, v);
  }
  s.mean = latencies_.empty() ? 0.0 : sum / (double)latencies_.size();
  s.max = mx;
  return s;
}

bool Scheduler::idle() {
  std::lock_guard<std::mutex> lk(mu_);
  if (!queue_.empty() || !ready_.empty()) return false;
  for (auto& b : running_)
    if (!b.empty()) return false;
  return true;
}

}  // namespace serve
}  // namespace stag
