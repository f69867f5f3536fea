// Request server: continuous batching of likelihood requests against resident datasets.
//
// Walker threads call tda_server_submit (never blocks on the GPU).  A scheduler
// thread takes, per dataset, the pending requests in arrival order up to max_batch
// templates, builds one row table of their template rows (no copy of the templates),
// and runs one batched evaluation of every dataset with pending work on a free slot
// (own stream and workspace).  A completion thread retires slots in launch order,
// stamps latencies and frees the slot for the next batch.  Up to n_slots batches are
// in flight, so new requests are admitted while earlier ones run.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "tda_internal.h"

using namespace tda;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket;
  int32_t ds;
  const double *H;
  int64_t B, ldh;
  double *out;
  double t_submit;
};

struct Dataset {
  tda_handle h;
  const double *d;
  int64_t N;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  MultiCtx *mc = nullptr;
  // device tables: row pointers, result staging, scatter descriptors
  void *rows_dev = nullptr;
  size_t rows_cap = 0;
  double *out_dev = nullptr;
  size_t out_cap = 0;
  int64_t *desc_dev = nullptr;
  size_t desc_cap = 0;
  // pinned host staging for the tables
  void *rows_host = nullptr;
  size_t rows_host_cap = 0;
  int64_t *desc_host = nullptr;
  size_t desc_host_cap = 0;
  std::vector<Request> reqs;
  bool busy = false;
  double t_launch = 0;
};

hipError_t grow_host(void **p, size_t *cap, size_t need) {
  if (need <= *cap) return hipSuccess;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  size_t c = std::max(need * 2, (size_t)4096);
  hipError_t e = hipHostMalloc(p, c, 0);
  if (e == hipSuccess) *cap = c;
  return e;
}

hipError_t grow_dev(void **p, size_t *cap, size_t need) {
  if (need <= *cap) return hipSuccess;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  size_t c = std::max(need * 2, (size_t)4096);
  hipError_t e = hipMalloc(p, c);
  if (e == hipSuccess) *cap = c;
  return e;
}

}  // namespace

struct tda_server {
  tda_server_options opt{};
  int device = 0;
  std::vector<Dataset> ds;
  size_t ds_bytes = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> pending;
  std::vector<Slot> slots;
  std::deque<int> inflight;
  std::vector<uint8_t> done;  // by ticket
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread sched, retire;
  // statistics
  std::vector<double> lat_ms;
  int64_t submitted = 0, completed = 0, rejected = 0, launches = 0, templates = 0, max_depth = 0;
  double busy_s = 0, busy_since = -1;
  tda_status error = TDA_OK;
  size_t slot_stage_bytes = 0;

  void scheduler();
  void retirer();
  tda_status launch(Slot &sl, std::vector<Request> &reqs, const std::vector<Dataset> &dsv);
};

tda_status tda_server::launch(Slot &sl, std::vector<Request> &reqs,
                              const std::vector<Dataset> &dsv) {
  // group by dataset in first-arrival order
  std::vector<int32_t> order;
  for (const Request &r : reqs)
    if (std::find(order.begin(), order.end(), r.ds) == order.end()) order.push_back(r.ds);
  std::vector<tda_work> items;
  std::vector<int64_t> row_off;  // per item offset into the row table
  std::vector<int64_t> out_off;
  int64_t rows = 0;
  for (int32_t d : order) {
    int64_t B = 0;
    for (const Request &r : reqs)
      if (r.ds == d) B += r.B;
    tda_work w{};
    w.h = dsv[d].h;
    w.d = dsv[d].d;
    w.H = nullptr;
    w.B = B;
    w.ldh = dsv[d].N;
    items.push_back(w);
    row_off.push_back(rows);
    out_off.push_back(rows);
    rows += B;
  }
  if (grow_dev(&sl.rows_dev, &sl.rows_cap, rows * sizeof(void *)) != hipSuccess ||
      grow_dev((void **)&sl.out_dev, &sl.out_cap, rows * sizeof(double)) != hipSuccess ||
      grow_dev((void **)&sl.desc_dev, &sl.desc_cap, reqs.size() * 3 * sizeof(int64_t)) !=
          hipSuccess)
    return set_error(TDA_ENOMEM, "server: staging allocation failed");
  // the slot's previous launch has retired, so its pinned tables are free to reuse
  if (grow_host(&sl.rows_host, &sl.rows_host_cap, std::max<size_t>(rows, 1) * sizeof(void *)) !=
          hipSuccess ||
      grow_host((void **)&sl.desc_host, &sl.desc_host_cap,
                std::max<size_t>(reqs.size(), 1) * 3 * sizeof(int64_t)) != hipSuccess)
    return set_error(TDA_ENOMEM, "server: pinned staging allocation failed");
  const double **rt = (const double **)sl.rows_host;
  std::vector<int64_t> fill(order.size(), 0);
  size_t nd = 0;
  for (const Request &r : reqs) {
    const size_t k = std::find(order.begin(), order.end(), r.ds) - order.begin();
    const int64_t base = row_off[k] + fill[k];
    for (int64_t b = 0; b < r.B; ++b) rt[base + b] = r.H + b * r.ldh;
    sl.desc_host[3 * nd] = (int64_t)(intptr_t)r.out;
    sl.desc_host[3 * nd + 1] = out_off[k] + fill[k];
    sl.desc_host[3 * nd + 2] = r.B;
    ++nd;
    fill[k] += r.B;
  }
  if (hipMemcpyAsync(sl.rows_dev, sl.rows_host, rows * sizeof(void *), hipMemcpyHostToDevice,
                     sl.stream) != hipSuccess ||
      hipMemcpyAsync(sl.desc_dev, sl.desc_host, nd * 3 * sizeof(int64_t), hipMemcpyHostToDevice,
                     sl.stream) != hipSuccess)
    return set_error(TDA_EHIP, "server: table upload failed");
  std::vector<const double *const *> hrows(items.size());
  for (size_t k = 0; k < items.size(); ++k) {
    hrows[k] = (const double *const *)sl.rows_dev + row_off[k];
    items[k].out = sl.out_dev + out_off[k];
  }
  tda_status st = multi_eval(sl.mc, items.data(), hrows.data(), (int64_t)items.size(),
                             opt.precision, sl.stream);
  if (st != TDA_OK) return st;
  if (launch_scatter(sl.desc_dev, (int64_t)nd, sl.out_dev, sl.stream) != hipSuccess)
    return set_error(TDA_EHIP, "server: scatter launch failed");
  if (hipEventRecord(sl.ev, sl.stream) != hipSuccess)
    return set_error(TDA_EHIP, "server: event record failed");
  return TDA_OK;
}

void tda_server::scheduler() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    int free_slot = -1;
    // wake for: work and a free slot, or shutdown with nothing left to launch
    cv.wait(lk, [&] {
      if (stop && pending.empty()) return true;
      if (pending.empty()) return false;
      for (size_t k = 0; k < slots.size(); ++k)
        if (!slots[k].busy) return true;
      return false;
    });
    if (stop && pending.empty()) return;
    for (size_t k = 0; k < slots.size(); ++k)
      if (!slots[k].busy) {
        free_slot = (int)k;
        break;
      }
    if (free_slot < 0) continue;
    // coalesce: per dataset, arrival order, up to max_batch templates (a request is
    // never split; an oversized request goes alone); stop at the slot's staging cap
    std::vector<Request> take;
    std::vector<int64_t> per_ds(ds.size(), 0);
    size_t stage = 0;
    std::deque<Request> keep;
    while (!pending.empty()) {
      Request r = pending.front();
      pending.pop_front();
      const int64_t cur = per_ds[r.ds];
      const size_t add = (size_t)r.B * (sizeof(void *) + sizeof(double));
      const bool fits_ds = cur == 0 || cur + r.B <= opt.max_batch;
      const bool fits_stage = take.empty() || stage + add <= slot_stage_bytes;
      if (fits_ds && fits_stage) {
        per_ds[r.ds] += r.B;
        stage += add;
        take.push_back(r);
      } else {
        keep.push_back(r);
      }
    }
    pending.swap(keep);
    Slot &sl = slots[free_slot];
    sl.busy = true;
    const std::vector<Dataset> dsv = ds;
    lk.unlock();
    tda_status st = launch(sl, take, dsv);
    lk.lock();
    if (st != TDA_OK) {
      error = st;
      for (const Request &r : take) done[r.ticket] = 2;  // failed
      sl.busy = false;
      cv.notify_all();
      continue;
    }
    sl.reqs.swap(take);
    sl.t_launch = now_s();
    if (busy_since < 0) busy_since = sl.t_launch;
    launches += 1;
    for (const Request &r : sl.reqs) templates += r.B;
    inflight.push_back(free_slot);
    cv.notify_all();
  }
}

void tda_server::retirer() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv.wait(lk, [&] { return !inflight.empty() || (stop && pending.empty()); });
    if (inflight.empty()) {
      bool any_busy = false;
      for (auto &s : slots) any_busy |= s.busy;
      if (stop && pending.empty() && !any_busy) return;
      continue;
    }
    const int k = inflight.front();
    Slot &sl = slots[k];
    lk.unlock();
    const hipError_t e = hipEventSynchronize(sl.ev);
    const double t = now_s();
    lk.lock();
    inflight.pop_front();
    for (const Request &r : sl.reqs) {
      done[r.ticket] = e == hipSuccess ? 1 : 2;
      lat_ms.push_back((t - r.t_submit) * 1e3);
      completed += 1;
    }
    sl.reqs.clear();
    sl.busy = false;
    if (inflight.empty() && busy_since >= 0) {
      busy_s += t - busy_since;
      busy_since = -1;
    }
    cv.notify_all();
  }
}

extern "C" tda_status tda_server_create(const tda_server_options *opt, tda_server_t *out) {
  if (!opt || !out) return set_error(TDA_EINVAL, "NULL argument");
  if (opt->struct_size < sizeof(tda_server_options)) return set_error(TDA_EINVAL, "struct_size");
  if (opt->n_slots < 1 || opt->n_slots > 16 || opt->max_batch < 1 || opt->max_queue < 1)
    return set_error(TDA_EINVAL, "n_slots in [1,16], max_batch >= 1, max_queue >= 1");
  if (opt->precision != TDA_PREC_FP64 && opt->precision != TDA_PREC_MIXED &&
      opt->precision != TDA_PREC_GS)
    return set_error(TDA_EINVAL, "unknown precision");
  *out = nullptr;
  tda_server *s = new tda_server();
  s->opt = *opt;
  s->device = opt->device;
  if (s->device < 0) (void)hipGetDevice(&s->device);
  (void)hipSetDevice(s->device);
  s->slot_stage_bytes = std::max<size_t>(opt->staging_bytes / opt->n_slots, 1 << 16);
  s->slots.resize(opt->n_slots);
  for (Slot &sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      delete s;
      return set_error(TDA_EHIP, "server: stream/event creation failed");
    }
    sl.mc = multi_ctx_create();
  }
  s->done.resize(1, 0);
  s->sched = std::thread([s] { s->scheduler(); });
  s->retire = std::thread([s] { s->retirer(); });
  *out = s;
  return TDA_OK;
}

extern "C" tda_status tda_server_add_dataset(tda_server_t s, tda_handle h, const double *d,
                                             int32_t *dataset) {
  if (!s || !h || !d || !dataset) return set_error(TDA_EINVAL, "NULL argument");
  if (handle_device(h) != s->device) return set_error(TDA_EINVAL, "dataset on another device");
  if (!handle_ready(h, s->opt.precision))
    return set_error(TDA_ESTATE, "dataset handle not factored for the server precision");
  std::lock_guard<std::mutex> lk(s->mu);
  const size_t bytes = handle_bytes(h);
  if (s->opt.dataset_budget_bytes && s->ds_bytes + bytes > s->opt.dataset_budget_bytes)
    return set_error(TDA_ENOMEM, "dataset budget exceeded");
  // whiten the data once, on the first slot's stream, before any request uses it
  (void)hipSetDevice(s->device);
  tda_status st = handle_set_data(h, d, s->slots[0].stream);
  if (st != TDA_OK) return st;
  if (hipStreamSynchronize(s->slots[0].stream) != hipSuccess)
    return set_error(TDA_EHIP, "server: data whitening failed");
  s->ds_bytes += bytes;
  s->ds.push_back(Dataset{h, d, handle_n(h)});
  *dataset = (int32_t)s->ds.size() - 1;
  return TDA_OK;
}

extern "C" tda_status tda_server_submit(tda_server_t s, int32_t dataset, const double *H,
                                        int64_t B, int64_t ldh, double *out, uint64_t *ticket) {
  if (!s || !ticket) return set_error(TDA_EINVAL, "NULL argument");
  const double t = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (dataset < 0 || dataset >= (int32_t)s->ds.size()) return set_error(TDA_EINVAL, "bad dataset");
  if (B < 1 || !H || !out || ldh < s->ds[dataset].N) return set_error(TDA_EINVAL, "bad request");
  if (s->stop) return set_error(TDA_ESTATE, "server stopping");
  if ((int64_t)s->pending.size() >= s->opt.max_queue ||
      (size_t)B * (sizeof(void *) + sizeof(double)) > s->slot_stage_bytes) {
    s->rejected += 1;
    return TDA_EAGAIN;
  }
  const uint64_t tk = s->next_ticket++;
  if (s->done.size() <= tk) s->done.resize(tk + 1, 0);
  s->pending.push_back(Request{tk, dataset, H, B, ldh, out, t});
  s->submitted += 1;
  s->max_depth = std::max<int64_t>(s->max_depth, (int64_t)s->pending.size());
  *ticket = tk;
  s->cv.notify_all();
  return TDA_OK;
}

extern "C" tda_status tda_server_poll(tda_server_t s, uint64_t ticket, int32_t *done) {
  if (!s || !done) return set_error(TDA_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return set_error(TDA_EINVAL, "unknown ticket");
  if (s->done[ticket] == 2) return set_error(TDA_EHIP, "request failed");
  *done = s->done[ticket] == 1;
  return TDA_OK;
}

extern "C" tda_status tda_server_wait(tda_server_t s, uint64_t ticket, double timeout_s) {
  if (!s) return set_error(TDA_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return set_error(TDA_EINVAL, "unknown ticket");
  const bool ok = s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                 [&] { return s->done[ticket] != 0; });
  if (!ok) return TDA_EAGAIN;
  return s->done[ticket] == 1 ? TDA_OK : set_error(TDA_EHIP, "request failed");
}

extern "C" tda_status tda_server_stats(tda_server_t s, tda_server_stats_t *st, int32_t reset) {
  if (!s || !st) return set_error(TDA_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(st, 0, sizeof *st);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->rejected = s->rejected;
  st->launches = s->launches;
  st->templates = s->templates;
  st->max_queue_depth = s->max_depth;
  st->busy_s = s->busy_s + (s->busy_since >= 0 ? now_s() - s->busy_since : 0.0);
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const double x = p / 100.0 * (double)(v.size() - 1);
      const size_t i = (size_t)x;
      const double f = x - (double)i;
      return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
    };
    st->p50_ms = pct(50);
    st->p99_ms = pct(99);
    double sum = 0;
    for (double x : v) sum += x;
    st->mean_ms = sum / (double)v.size();
    st->max_ms = v.back();
  }
  st->mean_templates_per_launch = s->launches ? (double)s->templates / (double)s->launches : 0;
  if (reset) {
    s->lat_ms.clear();
    s->submitted = s->completed = s->rejected = s->launches = s->templates = s->max_depth = 0;
    s->busy_s = 0;
    if (s->busy_since >= 0) s->busy_since = now_s();
  }
  return TDA_OK;
}

extern "C" tda_status tda_server_destroy(tda_server_t s) {
  if (!s) return TDA_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->sched.joinable()) s->sched.join();
  s->cv.notify_all();
  if (s->retire.joinable()) s->retire.join();
  (void)hipSetDevice(s->device);
  for (Slot &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    multi_ctx_destroy(sl.mc);
    if (sl.rows_dev) (void)hipFree(sl.rows_dev);
    if (sl.out_dev) (void)hipFree(sl.out_dev);
    if (sl.desc_dev) (void)hipFree(sl.desc_dev);
    if (sl.rows_host) (void)hipHostFree(sl.rows_host);
    if (sl.desc_host) (void)hipHostFree(sl.desc_host);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete s;
  return TDA_OK;
}
