// Serving loop on the GPU: resident data sets (prepared operands stay in HBM)
// and the continuous-batching scheduler of serve_core.h driving a GPU
// executor.  A batch packs the queries of several requests for one data set
// (each request padded to whole query tiles) into one operand set, runs one
// exact tile launch over it and one reduction that writes every request's
// results; batches of different data sets or streams overlap on the device.
// A query's value depends only on its own row and the data set, so a result
// is bitwise the same whether its request ran alone or in a mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "kde_exact.h"
#include "runtime.h"
#include "serve_core.h"

namespace stag {
namespace {

struct ReqSeg {
  int64_t row0;
  int64_t m;
  double* S;
};

__global__ void serve_reduce(const double* __restrict__ partial, int P, int64_t m_pad, const ReqSeg* __restrict__ segs,
                             int nseg) {
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
  double s = 0.0;
  for (int p = 0; p < P; ++p) s += partial[(int64_t)p * m_pad + row];
  segs[lo].S[local] = s;
}

struct Dataset {
  Operands xo;
  std::vector<void*> owned;
  int form = 0, d = 0;
  double a = 0.0;
  int64_t n = 0;
  int P = 0;
};

class GpuExecutor : public serve::Executor {
 public:
  GpuExecutor(int n_streams, int max_segs) : max_segs_(max_segs) {
    streams_.resize(n_streams, nullptr);
    events_.resize(n_streams, nullptr);
    pinned_.resize(n_streams, nullptr);
    bufs_.resize(n_streams);
    launched_.assign(n_streams, false);
    t0_ = std::chrono::steady_clock::now();
  }
  ~GpuExecutor() override {
    for (size_t s = 0; s < streams_.size(); ++s) {
      if (streams_[s]) (void)hipStreamSynchronize(streams_[s]);
      if (events_[s]) (void)hipEventDestroy(events_[s]);
      if (pinned_[s]) (void)hipHostFree(pinned_[s]);
      if (streams_[s]) (void)hipStreamDestroy(streams_[s]);
    }
    for (auto& ds : datasets_)
      for (void* p : ds->owned) (void)hipFree(p);
  }
  stag_status init() {
    for (size_t s = 0; s < streams_.size(); ++s) {
      STAG_HIP(hipStreamCreateWithFlags(&streams_[s], hipStreamNonBlocking));
      STAG_HIP(hipEventCreateWithFlags(&events_[s], hipEventDisableTiming));
      STAG_HIP(hipHostMalloc(reinterpret_cast<void**>(&pinned_[s]), sizeof(ReqSeg) * max_segs_));
    }
    return STAG_OK;
  }
  stag_status add_dataset(const float* X, int64_t n, int d, double a, int form, int* id) {
    std::unique_ptr<Dataset> ds(new Dataset());
    ds->form = form;
    ds->d = d;
    ds->a = a;
    ds->n = n;
    hipStream_t st = streams_[0];
    {
      Workspace ws(st);
      STAG_TRY(prepare_operands(form, X, n, d, a, false, ws, &ds->xo, st));
      ds->owned = ws.release();
    }
    STAG_HIP(hipStreamSynchronize(st));
    ds->P = (int)exact_chunks(ds->xo.rows_pad);
    *id = (int)datasets_.size();
    datasets_.push_back(std::move(ds));
    return STAG_OK;
  }
  int n_streams() const override { return (int)streams_.size(); }
  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }
  size_t footprint(int dsi, int64_t m) override {
    if (dsi < 0 || dsi >= (int)datasets_.size()) return 0;
    const Dataset& ds = *datasets_[dsi];
    const int64_t mp = round_up(m, query_tile_rows());
    const size_t per_row = (size_t)ds.xo.dp * form_element_bytes(ds.form) * form_parts(ds.form) + 4 + 8 +
                           (size_t)ds.P * 8;
    return (size_t)mp * per_row;
  }
  int launch(int dsi, const std::vector<serve::Request*>& batch, int s) override {
    const Dataset& ds = *datasets_[dsi];
    hipStream_t st = streams_[s];
    if ((int)batch.size() > max_segs_) return fail(STAG_E_INVAL, "serve: batch exceeds the segment table");
    int64_t total = 0;
    for (size_t k = 0; k < batch.size(); ++k) {
      pinned_[s][k] = ReqSeg{total, batch[k]->m, static_cast<double*>(batch[k]->S)};
      total += round_up(batch[k]->m, query_tile_rows());
    }
    Operands qo;
    qo.form = ds.form;
    qo.rows = total;
    qo.rows_pad = total;
    qo.d = ds.d;
    qo.dp = ds.xo.dp;
    auto& bufs = bufs_[s];
    bufs.clear();
    auto alloc = [&](void** p, size_t bytes) -> stag_status {
      hipError_t e = hipMallocAsync(p, std::max<size_t>(bytes, 256), st);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? STAG_E_NOMEM : STAG_E_DEVICE, "serve: workspace: %s",
                    hipGetErrorString(e));
      }
      bufs.push_back(*p);
      return STAG_OK;
    };
    stag_status rc = STAG_OK;
    auto release = [&]() {
      for (void* p : bufs) (void)hipFreeAsync(p, st);
      bufs.clear();
    };
    for (int p = 0; p < form_parts(ds.form) && rc == STAG_OK; ++p)
      rc = alloc(&qo.part[p], (size_t)total * qo.dp * form_element_bytes(ds.form));
    void* v = nullptr;
    if (rc == STAG_OK) rc = alloc(&v, (size_t)total * sizeof(float));
    qo.off = static_cast<float*>(v);
    if (rc == STAG_OK) rc = alloc(&v, (size_t)total * sizeof(double));
    qo.nrm = static_cast<double*>(v);
    double* partial = nullptr;
    if (rc == STAG_OK) rc = alloc(&v, (size_t)ds.P * total * sizeof(double));
    partial = static_cast<double*>(v);
    ReqSeg* dsegs = nullptr;
    if (rc == STAG_OK) rc = alloc(&v, sizeof(ReqSeg) * batch.size());
    dsegs = static_cast<ReqSeg*>(v);
    if (rc == STAG_OK)
      for (size_t k = 0; k < batch.size() && rc == STAG_OK; ++k)
        rc = prep_query_into(ds.form, static_cast<const float*>(batch[k]->Q), batch[k]->m, ds.d, ds.a, qo,
                             pinned_[s][k].row0, st);
    if (rc == STAG_OK) rc = launch_exact_tiles(ds.xo, qo, partial, TileExtra{}, st);
    if (rc == STAG_OK) {
      hipError_t e = hipMemcpyAsync(dsegs, pinned_[s], sizeof(ReqSeg) * batch.size(), hipMemcpyHostToDevice, st);
      if (e != hipSuccess) rc = fail(STAG_E_DEVICE, "serve: segment upload: %s", hipGetErrorString(e));
    }
    if (rc == STAG_OK) {
      ScopedTimer tm("serve_reduce", st);
      hipLaunchKernelGGL(serve_reduce, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, partial, ds.P, total,
                         dsegs, (int)batch.size());
      rc = check_launch("serve_reduce");
    }
    release();
    if (rc == STAG_OK) {
      hipError_t e = hipEventRecord(events_[s], st);
      if (e != hipSuccess) rc = fail(STAG_E_DEVICE, "serve: event: %s", hipGetErrorString(e));
    }
    if (rc != STAG_OK) {
      (void)hipStreamSynchronize(st);
      return rc;
    }
    launched_[s] = true;
    return STAG_OK;
  }
  bool finished(int s) override {
    if (!launched_[s]) return true;
    return hipEventQuery(events_[s]) != hipErrorNotReady;
  }
  std::vector<int> retire(int s) override {
    hipError_t e = hipEventSynchronize(events_[s]);
    launched_[s] = false;
    const int stt = e == hipSuccess ? STAG_OK : STAG_E_DEVICE;
    return std::vector<int>(1024, stt);
  }
  int n_datasets() const { return (int)datasets_.size(); }

 private:
  int max_segs_;
  std::vector<hipStream_t> streams_;
  std::vector<hipEvent_t> events_;
  std::vector<ReqSeg*> pinned_;
  std::vector<std::vector<void*>> bufs_;
  std::vector<bool> launched_;
  std::vector<std::unique_ptr<Dataset>> datasets_;
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
                               stag_server** out) {
  using namespace stag;
  if (!out) return fail(STAG_E_INVAL, "stag_server_create: out is NULL");
  *out = nullptr;
  if (n_streams < 0 || n_streams > 16) return fail(STAG_E_INVAL, "stag_server_create: n_streams must be in [0, 16]");
  if (max_batch_queries < 0) return fail(STAG_E_INVAL, "stag_server_create: max_batch_queries must be >= 0");
  clear_error();
  std::unique_ptr<stag_server> sv(new stag_server());
  const int ns = n_streams > 0 ? n_streams : 4;
  const int64_t mb = max_batch_queries > 0 ? max_batch_queries : 65536;
  sv->ex.reset(new GpuExecutor(ns, 1024));
  STAG_TRY(sv->ex->init());
  STAG_HIP(hipGetDevice(&sv->device));
  sv->sched.reset(new serve::Scheduler(sv->ex.get(), budget_bytes > 0 ? budget_bytes : ((size_t)8 << 30), mb));
  *out = sv.release();
  return STAG_OK;
}

stag_status stag_server_add_dataset(stag_server* s, const float* X, int64_t n, int32_t d, double a, int32_t form,
                                    int32_t* id_out) {
  using namespace stag;
  if (!s || !X || !id_out) return fail(STAG_E_INVAL, "stag_server_add_dataset: NULL argument");
  if (n < 1 || d < 1 || !(a > 0.0) || !std::isfinite(a))
    return fail(STAG_E_INVAL, "stag_server_add_dataset: need n, d >= 1 and finite a > 0");
  if (form < STAG_FORM_FP32 || form > STAG_FORM_BF16_SPLIT3)
    return fail(STAG_E_INVAL, "stag_server_add_dataset: unknown form %d", form);
  if (exact_padded_dim(d) == 0 || (d > 256 && form != STAG_FORM_FP32))
    return fail(STAG_E_UNSUPPORTED, "stag_server_add_dataset: d = %d not supported by this form", d);
  clear_error();
  // the scheduler's worker thread must not run while a data set is added
  s->sched->stop();
  int id = 0;
  const stag_status st = s->ex->add_dataset(X, n, d, a, form, &id);
  if (st == STAG_OK) *id_out = id;
  return st;
}

stag_status stag_server_submit(stag_server* s, int32_t dataset, const float* Q, int64_t m, double* S_out,
                               uint64_t* ticket) {
  using namespace stag;
  if (!s || !Q || !S_out || !ticket) return fail(STAG_E_INVAL, "stag_server_submit: NULL argument");
  if (dataset < 0 || dataset >= s->ex->n_datasets()) return fail(STAG_E_INVAL, "stag_server_submit: bad data set");
  if (m < 1) return fail(STAG_E_INVAL, "stag_server_submit: m must be >= 1");
  *ticket = s->sched->submit(dataset, Q, m, S_out);
  if (*ticket == 0) return fail(STAG_E_INVAL, "stag_server_submit: rejected");
  s->sched->start();
  return STAG_OK;
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
