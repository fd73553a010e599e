// Serving loop on the GPU: resident data sets and CKNS indexes, and the
// continuous-batching scheduler of serve_core.h driving a GPU executor.
//
// A data set keeps X prepared in HBM in each of its resident exact forms
// (the fp32 form with its tiles centred, the split forms as hi/lo parts) and,
// optionally, a CKNS index.  A request is an exact request in one resident
// form (given, or chosen per request from its eps by the STAG_FORM_AUTO rule
// at submission) or an LSH request answered by the resident index.  The
// scheduler batches chunks of requests with the same data set and key (the
// form, or the index).  Each stream has a host worker thread that issues its
// batches:
//   exact  the chunks' queries are prepared into one operand set (each chunk
//          padded to whole query tiles), one tile launch covers them and one
//          segmented reduction writes every chunk's results (and bounds);
//   lsh    one index query per chunk (the query synchronises once with the
//          host for its task count, which is why it runs on the worker).
// Batches of different streams overlap on the device.  A query's value
// depends only on its own row and the data set, so a result is bitwise the
// same whether its request ran alone, chunked, or in a mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "kde_exact.h"
#include "runtime.h"
#include "serve_core.h"

namespace stag {
namespace {

constexpr int kKeyLsh = 100;           // batching key of LSH requests (exact: the form)
constexpr int kMaxItems = 1024;        // items (request chunks) per batch
constexpr int64_t kQueryTile = 128;    // queries per tile of the exact kernels

struct ReqSeg {
  int64_t row0;  // first row of the chunk in the batch operand set
  int64_t m;     // rows of the chunk
  double* S;
  double* B;
};

// Segmented reduction of one exact batch: S (and the bound) of every chunk.
// Centred data (bpart != null): bound = (sum bpart) / S; else the a-priori
// bound at the query's norm and the data set's largest norm.
__global__ void serve_reduce(const double* __restrict__ partial, const double* __restrict__ bpart, int P,
                             int64_t m_pad, const ReqSeg* __restrict__ segs, int nseg,
                             const double* __restrict__ qnrm, const unsigned long long* __restrict__ max_xnrm_bits,
                             BoundModel bm) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= m_pad) return;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {  // last segment with row0 <= row
    const int mid = (lo + hi + 1) / 2;
    if (segs[mid].row0 <= row) lo = mid;
    else hi = mid - 1;
  }
  const int64_t local = row - segs[lo].row0;
  if (local < 0 || local >= segs[lo].m) return;
  const double s = chunk_sum(partial + row, P, m_pad);
  segs[lo].S[local] = s;
  if (segs[lo].B) {
    if (bpart) {
      const double b = chunk_sum(bpart + row, P, m_pad);
      const double r = b / s;
      segs[lo].B[local] = s > 0.0 ? r + r * r + bm.c_tail : HUGE_VAL;
    } else {
      segs[lo].B[local] = relative_bound(bm, qnrm[row], __longlong_as_double((long long)*max_xnrm_bits));
    }
  }
}

struct Dataset {
  int64_t n = 0;
  int d = 0;
  double a = 0.0;
  uint32_t forms = 0;  // resident exact forms (1 << form)
  Operands ops[4];
  std::vector<void*> owned;
  double max_nrm_x = 0.0;
  float max_abs_x = 0.0f;
  stag_lsh_index* lsh = nullptr;
  stag_lsh_shape lsh_shape{};
};

// A host thread per stream that runs that stream's batch launches.
class Worker {
 public:
  Worker() : th_([this] { loop(); }) {}
  ~Worker() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    th_.join();
  }
  void post(std::function<int()> f) {
    std::lock_guard<std::mutex> lk(mu_);
    task_ = std::move(f);
    done_ = false;
    has_ = true;
    cv_.notify_all();
  }
  bool done() const { return done_.load(std::memory_order_acquire); }
  int wait() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return done_.load(); });
    return rc_;
  }

 private:
  void loop() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || has_; });
      if (stop_ && !has_) return;
      std::function<int()> f = std::move(task_);
      has_ = false;
      lk.unlock();
      const int rc = f();
      lk.lock();
      rc_ = rc;
      done_.store(true, std::memory_order_release);
      cv_done_.notify_all();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  std::function<int()> task_;
  bool has_ = false, stop_ = false;
  std::atomic<bool> done_{true};
  int rc_ = 0;
  std::thread th_;
};

class GpuExecutor : public serve::Executor {
 public:
  explicit GpuExecutor(int n_streams) {
    streams_.resize(n_streams, nullptr);
    events_.resize(n_streams, nullptr);
    pinned_.resize(n_streams, nullptr);
    launched_.assign(n_streams, false);
    t0_ = std::chrono::steady_clock::now();
  }
  ~GpuExecutor() override {
    workers_.clear();  // joins the threads (each finishes its task first)
    for (size_t s = 0; s < streams_.size(); ++s) {
      if (streams_[s]) (void)hipStreamSynchronize(streams_[s]);
      if (events_[s]) (void)hipEventDestroy(events_[s]);
      if (pinned_[s]) (void)hipHostFree(pinned_[s]);
      if (streams_[s]) (void)hipStreamDestroy(streams_[s]);
    }
    if (admin_) (void)hipStreamSynchronize(admin_);
    for (auto& ds : datasets_) {
      if (ds->lsh) stag_lsh_index_destroy(ds->lsh);
      for (void* p : ds->owned) (void)hipFree(p);
    }
    if (stat_dev_) (void)hipFree(stat_dev_);
    if (stat_host_) (void)hipHostFree(stat_host_);
    if (admin_) (void)hipStreamDestroy(admin_);
  }
  stag_status init() {
    for (size_t s = 0; s < streams_.size(); ++s) {
      STAG_HIP(hipStreamCreateWithFlags(&streams_[s], hipStreamNonBlocking));
      STAG_HIP(hipEventCreateWithFlags(&events_[s], hipEventDisableTiming));
      STAG_HIP(hipHostMalloc(reinterpret_cast<void**>(&pinned_[s]), sizeof(ReqSeg) * kMaxItems));
    }
    STAG_HIP(hipStreamCreateWithFlags(&admin_, hipStreamNonBlocking));
    STAG_HIP(hipMalloc(&stat_dev_, 256));
    STAG_HIP(hipHostMalloc(&stat_host_, 256));
    for (size_t s = 0; s < streams_.size(); ++s) workers_.emplace_back(new Worker());
    return STAG_OK;
  }

  // Largest squared row norm and |element| of A [rows][d] (device), waiting
  // on the admin stream.
  stag_status stats_of(const float* A, int64_t rows, int d, double* max_nrm, float* max_abs) {
    std::lock_guard<std::mutex> lk(admin_mu_);
    auto* nb = static_cast<unsigned long long*>(stat_dev_);
    auto* ab = reinterpret_cast<unsigned int*>(static_cast<char*>(stat_dev_) + 64);
    auto* bad = reinterpret_cast<int*>(static_cast<char*>(stat_dev_) + 128);
    STAG_TRY(row_stats_async(A, rows, d, nb, ab, bad, admin_));
    STAG_HIP(hipMemcpyAsync(stat_host_, stat_dev_, 192, hipMemcpyDeviceToHost, admin_));
    STAG_HIP(hipStreamSynchronize(admin_));
    std::memcpy(max_nrm, stat_host_, sizeof(double));
    std::memcpy(max_abs, static_cast<char*>(stat_host_) + 64, sizeof(float));
    return STAG_OK;
  }

  stag_status add_dataset(const float* X, int64_t n, int d, double a, uint32_t forms, double lsh_eps,
                          const stag_lsh_params* lsh, int* id) {
    std::unique_ptr<Dataset> ds(new Dataset());
    ds->n = n;
    ds->d = d;
    ds->a = a;
    ds->forms = forms;
    hipStream_t st = admin_;
    STAG_TRY(stats_of(X, n, d, &ds->max_nrm_x, &ds->max_abs_x));
    for (int f = 0; f < 4; ++f) {
      if (!(forms & (1u << f))) continue;
      Workspace ws(st);
      if (f == STAG_FORM_FP32 && exact_padded_dim(d) <= 256) {
        // fp32: centred tiles (the grouping's temporaries go back to the pool)
        Workspace tmp(st);
        CentreTemp t;
        STAG_TRY(alloc_centred_operands(n, d, ws, &ds->ops[f]));
        STAG_TRY(alloc_centre_temp(ds->ops[f], tmp, &t));
        STAG_TRY(prep_centred_operands(X, a, ds->ops[f], t, st));
        for (void* p : ws.release()) ds->owned.push_back(p);
      } else {
        STAG_TRY(prepare_operands(f, X, n, d, a, false, ws, &ds->ops[f], st));
        for (void* p : ws.release()) ds->owned.push_back(p);
      }
    }
    if (lsh) {
      STAG_TRY(stag_lsh_index_create(X, n, d, a, lsh_eps, lsh, &ds->lsh, st));
      STAG_TRY(stag_lsh_index_shape(ds->lsh, &ds->lsh_shape));
    }
    STAG_HIP(hipStreamSynchronize(st));
    *id = (int)datasets_.size();
    datasets_.push_back(std::move(ds));
    return STAG_OK;
  }

  int n_streams() const override { return (int)streams_.size(); }
  int max_batch_items() const override { return kMaxItems; }
  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }
  size_t footprint(int dsi, int key, int64_t m) override {
    if (dsi < 0 || dsi >= (int)datasets_.size()) return 0;
    const Dataset& ds = *datasets_[dsi];
    const int64_t mp = round_up(m, kQueryTile);
    if (key == kKeyLsh) {
      if (!ds.lsh) return 0;
      const stag_lsh_shape& sh = ds.lsh_shape;
      return (size_t)mp * ((size_t)sh.K1 * sh.J * sh.L * 16 + 64) + ((size_t)64 << 20);
    }
    if (key < 0 || key > 3 || !(ds.forms & (1u << key))) return 0;
    const Operands& xo = ds.ops[key];
    const int P = (int)exact_chunks(xo.rows_pad);
    const size_t per_row = (size_t)xo.dp * form_element_bytes(key) * form_parts(key) + 4 + 8 +
                           (size_t)P * 8 * (xo.centred ? 2 : 1);
    return (size_t)mp * per_row;
  }

  int launch(int dsi, int key, const std::vector<serve::Item>& batch, int s) override {
    if ((int)batch.size() > kMaxItems) return fail(STAG_E_INVAL, "serve: batch exceeds the segment table");
    const Dataset* ds = datasets_[dsi].get();
    hipStream_t st = streams_[s];
    hipEvent_t ev = events_[s];
    ReqSeg* pinned = pinned_[s];
    std::vector<serve::Item> items = batch;
    if (key == kKeyLsh) {
      workers_[s]->post([ds, items, st, ev]() -> int {
        int rc = STAG_OK;
        for (const serve::Item& it : items) {
          const float* Q = static_cast<const float*>(it.r->Q) + it.row0 * ds->d;
          double* S = static_cast<double*>(it.r->S) + it.row0;
          rc = stag_lsh_index_query(ds->lsh, Q, it.m, S, st);
          if (rc != STAG_OK) break;
        }
        if (hipEventRecord(ev, st) != hipSuccess && rc == STAG_OK) rc = STAG_E_DEVICE;
        if (rc != STAG_OK) (void)hipStreamSynchronize(st);
        return rc;
      });
    } else {
      workers_[s]->post([ds, key, items, st, ev, pinned]() -> int {
        const int rc = run_exact_batch(*ds, key, items, st, pinned);
        int rc2 = rc;
        if (hipEventRecord(ev, st) != hipSuccess && rc2 == STAG_OK) rc2 = STAG_E_DEVICE;
        if (rc2 != STAG_OK) (void)hipStreamSynchronize(st);
        return rc2;
      });
    }
    launched_[s] = true;
    return STAG_OK;
  }
  bool finished(int s) override {
    if (!launched_[s]) return true;
    if (!workers_[s]->done()) return false;
    return hipEventQuery(events_[s]) != hipErrorNotReady;
  }
  std::vector<int> retire(int s) override {
    int rc = workers_[s]->wait();
    if (rc == STAG_OK && hipEventSynchronize(events_[s]) != hipSuccess) rc = STAG_E_DEVICE;
    launched_[s] = false;
    return std::vector<int>(kMaxItems, rc);
  }
  int n_datasets() const { return (int)datasets_.size(); }
  const Dataset* dataset(int i) const { return datasets_[i].get(); }

 private:
  // One exact batch on stream st: chunk queries into one operand set, tiles,
  // segmented reduction.  Temporaries are stream-ordered pool allocations.
  static stag_status run_exact_batch(const Dataset& ds, int form, const std::vector<serve::Item>& items,
                                     hipStream_t st, ReqSeg* pinned) {
    const Operands& xo = ds.ops[form];
    const bool centred = xo.centred;
    int64_t total = 0;
    for (size_t k = 0; k < items.size(); ++k) {
      const serve::Item& it = items[k];
      double* B = it.r->B ? static_cast<double*>(it.r->B) + it.row0 : nullptr;
      pinned[k] = ReqSeg{total, it.m, static_cast<double*>(it.r->S) + it.row0, B};
      total += round_up(it.m, kQueryTile);
    }
    Operands qo;
    qo.form = form;
    qo.rows = total;
    qo.rows_pad = total;
    qo.d = ds.d;
    qo.dp = xo.dp;
    Workspace ws(st);
    for (int p = 0; p < form_parts(form); ++p)
      STAG_TRY(ws.alloc_bytes(&qo.part[p], (size_t)total * qo.dp * form_element_bytes(form)));
    STAG_TRY(ws.alloc(&qo.off, (size_t)total));
    STAG_TRY(ws.alloc(&qo.nrm, (size_t)total));
    const int P = (int)exact_chunks(xo.rows_pad);
    double *partial = nullptr, *bpart = nullptr;
    STAG_TRY(ws.alloc(&partial, (size_t)P * total));
    if (centred) STAG_TRY(ws.alloc(&bpart, (size_t)P * total));
    ReqSeg* dsegs = nullptr;
    STAG_TRY(ws.alloc(&dsegs, items.size()));
    for (size_t k = 0; k < items.size(); ++k) {
      const serve::Item& it = items[k];
      const float* Q = static_cast<const float*>(it.r->Q) + it.row0 * ds.d;
      STAG_TRY(prep_query_into(form, Q, it.m, ds.d, ds.a, qo, pinned[k].row0, st, centred));
    }
    const BoundModel bm = make_bound_model(form, ds.d, ds.a, STAG_KERNEL_GAUSSIAN);
    TileExtra ex;
    ex.a = ds.a;
    ex.bpart = bpart;
    ex.c_cent = (float)bm.c_cent;
    STAG_TRY(launch_exact_tiles(xo, qo, partial, ex, st));
    STAG_HIP(hipMemcpyAsync(dsegs, pinned, sizeof(ReqSeg) * items.size(), hipMemcpyHostToDevice, st));
    ScopedTimer tm("serve_reduce", st);
    hipLaunchKernelGGL(serve_reduce, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, partial, bpart, P, total,
                       dsegs, (int)items.size(), qo.nrm, xo.max_nrm_bits, bm);
    return check_launch("serve_reduce");
  }

  std::vector<hipStream_t> streams_;
  std::vector<hipEvent_t> events_;
  std::vector<ReqSeg*> pinned_;
  std::vector<bool> launched_;
  std::vector<std::unique_ptr<Worker>> workers_;
  std::vector<std::unique_ptr<Dataset>> datasets_;
  hipStream_t admin_ = nullptr;
  std::mutex admin_mu_;
  void* stat_dev_ = nullptr;
  void* stat_host_ = nullptr;
  std::chrono::steady_clock::time_point t0_;
};

}  // namespace
}  // namespace stag

struct stag_server {
  std::unique_ptr<stag::GpuExecutor> ex;
  std::unique_ptr<stag::serve::Scheduler> sched;
  int device = 0;
};

extern "C" {

stag_status stag_server_create(size_t budget_bytes, int32_t n_streams, int64_t max_batch_queries,
                               int64_t chunk_queries, stag_server** out) {
  using namespace stag;
  if (!out) return fail(STAG_E_INVAL, "stag_server_create: out is NULL");
  *out = nullptr;
  if (n_streams < 0 || n_streams > 16) return fail(STAG_E_INVAL, "stag_server_create: n_streams must be in [0, 16]");
  if (max_batch_queries < 0 || chunk_queries < 0)
    return fail(STAG_E_INVAL, "stag_server_create: max_batch_queries and chunk_queries must be >= 0");
  clear_error();
  std::unique_ptr<stag_server> sv(new stag_server());
  const int ns = n_streams > 0 ? n_streams : 4;
  const int64_t mb = max_batch_queries > 0 ? max_batch_queries : 65536;
  const int64_t ch = chunk_queries > 0 ? chunk_queries : 4096;
  sv->ex.reset(new GpuExecutor(ns));
  STAG_TRY(sv->ex->init());
  STAG_HIP(hipGetDevice(&sv->device));
  sv->sched.reset(new serve::Scheduler(sv->ex.get(), budget_bytes > 0 ? budget_bytes : ((size_t)8 << 30), mb, ch));
  *out = sv.release();
  return STAG_OK;
}

stag_status stag_server_add_dataset_ex(stag_server* s, const float* X, int64_t n, int32_t d, double a, uint32_t forms,
                                       double lsh_eps, const stag_lsh_params* lsh, int32_t* id_out) {
  using namespace stag;
  const char* fn = "stag_server_add_dataset_ex";
  if (!s || !X || !id_out) return fail(STAG_E_INVAL, "%s: NULL argument", fn);
  if (n < 1 || d < 1 || !(a > 0.0) || !std::isfinite(a))
    return fail(STAG_E_INVAL, "%s: need n, d >= 1 and finite a > 0", fn);
  if (forms & ~0xFu) return fail(STAG_E_INVAL, "%s: unknown form bits 0x%x", fn, forms);
  if (forms == 0 && !lsh) return fail(STAG_E_INVAL, "%s: neither an exact form nor an index", fn);
  if (exact_padded_dim(d) == 0 || (d > 256 && (forms & ~(1u << STAG_FORM_FP32))))
    return fail(STAG_E_UNSUPPORTED, "%s: d = %d not supported by these forms", fn, d);
  if (lsh && !(lsh_eps > 0.0 && lsh_eps < 1.0)) return fail(STAG_E_INVAL, "%s: lsh eps must be in (0, 1)", fn);
  clear_error();
  // the scheduler's worker thread must not run while a data set is added
  s->sched->stop();
  int id = 0;
  const stag_status st = s->ex->add_dataset(X, n, d, a, forms, lsh_eps, lsh, &id);
  if (st == STAG_OK) *id_out = id;
  return st;
}

stag_status stag_server_add_dataset(stag_server* s, const float* X, int64_t n, int32_t d, double a, int32_t form,
                                    int32_t* id_out) {
  using namespace stag;
  if (form < STAG_FORM_FP32 || form > STAG_FORM_BF16_SPLIT3)
    return fail(STAG_E_INVAL, "stag_server_add_dataset: unknown form %d", form);
  return stag_server_add_dataset_ex(s, X, n, d, a, 1u << form, 0.0, nullptr, id_out);
}

stag_status stag_server_submit_ex(stag_server* s, int32_t dataset, const float* Q, int64_t m, int32_t kind,
                                  int32_t form, double eps, double* S_out, double* bound_out, int32_t* form_out,
                                  uint64_t* ticket) {
  using namespace stag;
  const char* fn = "stag_server_submit_ex";
  if (!s || !Q || !S_out || !ticket) return fail(STAG_E_INVAL, "%s: NULL argument", fn);
  if (dataset < 0 || dataset >= s->ex->n_datasets()) return fail(STAG_E_INVAL, "%s: bad data set", fn);
  if (m < 1) return fail(STAG_E_INVAL, "%s: m must be >= 1", fn);
  const Dataset* ds = s->ex->dataset(dataset);
  int key = 0;
  if (kind == STAG_REQUEST_LSH) {
    if (!ds->lsh) return fail(STAG_E_INVAL, "%s: data set %d has no resident index", fn, dataset);
    if (bound_out) return fail(STAG_E_INVAL, "%s: LSH requests have no per-result bound", fn);
    key = kKeyLsh;
  } else if (kind == STAG_REQUEST_EXACT) {
    if (form == STAG_FORM_AUTO) {
      if (!(eps > 0.0)) return fail(STAG_E_INVAL, "%s: STAG_FORM_AUTO needs eps > 0", fn);
      double qn = 0.0;
      float qa = 0.0f;
      STAG_TRY(s->ex->stats_of(Q, m, ds->d, &qn, &qa));
      key = choose_resident_form(ds->forms, ds->d, ds->a, eps, qn, ds->max_nrm_x, qa, ds->max_abs_x);
      if (key < 0) return fail(STAG_E_INVAL, "%s: data set %d has no resident exact form", fn, dataset);
    } else {
      if (form < STAG_FORM_FP32 || form > STAG_FORM_BF16_SPLIT3 || !(ds->forms & (1u << form)))
        return fail(STAG_E_INVAL, "%s: form %d is not resident for data set %d", fn, form, dataset);
      key = form;
    }
  } else {
    return fail(STAG_E_INVAL, "%s: unknown request kind %d", fn, kind);
  }
  if (form_out) *form_out = key == kKeyLsh ? -1 : key;
  *ticket = s->sched->submit(dataset, key, Q, m, S_out, bound_out);
  if (*ticket == 0) return fail(STAG_E_INVAL, "%s: rejected", fn);
  s->sched->start();
  return STAG_OK;
}

stag_status stag_server_submit(stag_server* s, int32_t dataset, const float* Q, int64_t m, double* S_out,
                               uint64_t* ticket) {
  using namespace stag;
  if (!s) return fail(STAG_E_INVAL, "stag_server_submit: NULL server");
  if (dataset < 0 || dataset >= s->ex->n_datasets()) return fail(STAG_E_INVAL, "stag_server_submit: bad data set");
  const uint32_t forms = s->ex->dataset(dataset)->forms;
  int form = 0;
  while (form < 4 && !(forms & (1u << form))) ++form;
  if (form == 4) return fail(STAG_E_INVAL, "stag_server_submit: data set %d has no resident exact form", dataset);
  return stag_server_submit_ex(s, dataset, Q, m, STAG_REQUEST_EXACT, form, 0.0, S_out, nullptr, nullptr, ticket);
}

stag_status stag_server_wait(stag_server* s, uint64_t ticket, stag_status* result, double* latency_s) {
  using namespace stag;
  if (!s) return fail(STAG_E_INVAL, "stag_server_wait: NULL server");
  s->sched->start();
  const int st = s->sched->wait(ticket, latency_s);
  if (result) *result = (stag_status)st;
  return STAG_OK;
}

stag_status stag_server_poll(stag_server* s, uint64_t ticket, int32_t* done, stag_status* result,
                             double* latency_s) {
  using namespace stag;
  if (!s || !done) return fail(STAG_E_INVAL, "stag_server_poll: NULL argument");
  int st = 0;
  const int r = s->sched->poll(ticket, &st, latency_s);
  if (r < 0) return fail(STAG_E_INVAL, "stag_server_poll: unknown ticket");
  *done = r;
  if (result && r == 1) *result = (stag_status)st;
  return STAG_OK;
}

stag_status stag_server_stats(stag_server* s, stag_server_stats_t* out) {
  using namespace stag;
  if (!s || !out) return fail(STAG_E_INVAL, "stag_server_stats: NULL argument");
  const serve::Stats st = s->sched->stats();
  out->submitted = st.submitted;
  out->completed = st.completed;
  out->failed = st.failed;
  out->rejected = st.rejected;
  out->batches = st.batches;
  out->queries = st.queries;
  out->p50_s = st.p50;
  out->p99_s = st.p99;
  out->mean_s = st.mean;
  out->max_s = st.max;
  out->inflight_bytes = st.inflight_bytes;
  out->peak_inflight_bytes = st.peak_inflight_bytes;
  return STAG_OK;
}

void stag_server_destroy(stag_server* s) {
  if (!s) return;
  s->sched->stop();
  s->sched.reset();
  s->ex.reset();
  delete s;
}

}  // extern "C"
