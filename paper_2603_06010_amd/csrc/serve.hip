// Request server: continuous batching of likelihood requests against resident datasets.
//
// Walker threads call tda_server_submit (never blocks on the GPU).  A scheduler
// thread takes, per dataset, the pending requests in arrival order up to max_batch
// templates, builds one row table of their template rows (no copy of the templates),
// and runs one batched evaluation of every dataset with pending work on a free slot
// (own stream and workspace).  A completion thread retires slots in launch order,
// stamps latencies and frees the slot for the next batch.  Up to n_slots batches are
// in flight, so new requests are admitted while earlier ones run.
//
// Bounded bookkeeping: request states live in a ring indexed by ticket (sized at creation
// to hold every request that can be outstanding), latencies in a fixed log-spaced
// histogram, and each slot's device and pinned tables are sized at creation for the
// largest batch its staging share admits, so nothing grows while the server runs.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
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

// device memory left free when a launch's workspace is sized (descriptor rings, the
// runtime, other small allocations)
constexpr size_t kMemMargin = (size_t)1 << 30;

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
  // (sized at creation: rows_cap template rows, desc_cap requests)
  void *rows_dev = nullptr;
  size_t rows_cap = 0;
  double *out_dev = nullptr;
  int64_t *desc_dev = nullptr;
  size_t desc_cap = 0;
  // pinned host staging for the tables
  void *rows_host = nullptr;
  int64_t *desc_host = nullptr;
  std::vector<Request> reqs;
  bool busy = false;
  double t_launch = 0;
};

// Latency histogram: bucket k covers [kLatMin * kLatStep^k, kLatMin * kLatStep^(k+1)) ms,
// 1 us to about 1e5 s at 1 % resolution; the first and last buckets take what falls outside.
constexpr int kLatBuckets = 2560;
constexpr double kLatMin = 1e-3;
constexpr double kLatStep = 1.01;

struct LatencyHist {
  std::vector<int64_t> n = std::vector<int64_t>(kLatBuckets, 0);
  int64_t count = 0;
  double sum = 0.0, max = 0.0;
  void add(double ms) {
    int k = ms <= kLatMin ? 0 : (int)(log(ms / kLatMin) / log(kLatStep));
    k = std::min(std::max(k, 0), kLatBuckets - 1);
    n[k] += 1;
    count += 1;
    sum += ms;
    max = std::max(max, ms);
  }
  // p-th percentile, interpolated inside its bucket (geometrically)
  double pct(double p) const {
    if (count == 0) return 0.0;
    const double target = p / 100.0 * (double)count;
    int64_t below = 0;
    for (int k = 0; k < kLatBuckets; ++k) {
      if (n[k] == 0) continue;
      if ((double)(below + n[k]) >= target) {
        const double f = std::min(std::max((target - (double)below) / (double)n[k], 0.0), 1.0);
        return std::min(kLatMin * pow(kLatStep, (double)k + f), max);
      }
      below += n[k];
    }
    return max;
  }
  void clear() {
    std::fill(n.begin(), n.end(), 0);
    count = 0;
    sum = max = 0.0;
  }
};

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
  // request state by ticket: ring[t & ring_mask] = 0 pending, 1 done, 2 failed.  The ring
  // holds at least twice as many entries as requests can be outstanding (pending or in
  // flight), so a ticket older than one ring length has completed; failures of such old
  // tickets are kept in a short list.
  std::vector<uint8_t> ring;
  uint64_t ring_mask = 0;
  std::deque<uint64_t> old_failed;
  int64_t outstanding = 0;
  int64_t max_outstanding = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread sched, retire;
  // statistics
  LatencyHist lat;
  int64_t submitted = 0, completed = 0, rejected = 0, launches = 0, templates = 0, max_depth = 0;
  double busy_s = 0, busy_since = -1;
  tda_status error = TDA_OK;
  std::string error_msg;  // message of the last failed launch (the scheduler thread's)
  size_t slot_stage_bytes = 0;

  void scheduler();
  void retirer();
  uint8_t &state(uint64_t t) { return ring[t & ring_mask]; }
  // 0 pending, 1 done, 2 failed; ticket known to have been issued
  uint8_t status(uint64_t t) const {
    if (t + ring_mask + 1 > next_ticket) return ring[t & ring_mask];
    return std::find(old_failed.begin(), old_failed.end(), t) != old_failed.end() ? 2 : 1;
  }
  void finish(uint64_t t, uint8_t st) {
    ring[t & ring_mask] = st;
    if (st == 2) {
      old_failed.push_back(t);
      if (old_failed.size() > 4096) old_failed.pop_front();
    }
    outstanding -= 1;
  }
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
  // tables sized at creation for slot_rows templates (the coalescing never takes more);
  // the slot's previous launch has retired, so its pinned tables are free to reuse
  if ((size_t)rows > sl.rows_cap || reqs.size() > sl.desc_cap)
    return set_error(TDA_EINTERNAL, "server: batch beyond the slot tables");
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
    // never split; an oversized request goes alone); stop at the slot's staging cap and at
    // the device memory the launch's workspace may take: what is free now plus what this
    // slot's workspace already holds (reused or replaced), less a margin
    std::vector<Request> take;
    std::vector<int64_t> per_ds(ds.size(), 0);
    size_t stage = 0;
    size_t avail = SIZE_MAX, ws_items = 0, ws_fixed = 0;
    {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
        const size_t have = free_b + multi_ctx_held(slots[free_slot].mc);
        avail = have > kMemMargin ? have - kMemMargin : 0;
      }
      (void)hipGetLastError();
    }
    std::deque<Request> keep;
    while (!pending.empty()) {
      Request r = pending.front();
      pending.pop_front();
      const int64_t cur = per_ds[r.ds];
      const size_t add = (size_t)r.B * (sizeof(void *) + sizeof(double));
      const size_t w_old = item_ws_bytes(ds[r.ds].h, cur, opt.precision);
      const size_t w_new = item_ws_bytes(ds[r.ds].h, cur + r.B, opt.precision);
      const size_t fixed = std::max(ws_fixed, launch_ws_fixed_bytes(ds[r.ds].h, opt.precision));
      const bool fits_ds = cur == 0 || cur + r.B <= opt.max_batch;
      const bool fits_stage = take.empty() || stage + add <= slot_stage_bytes;
      const bool fits_mem = take.empty() || ws_items - w_old + w_new + fixed <= avail;
      if (fits_ds && fits_stage && fits_mem) {
        per_ds[r.ds] += r.B;
        stage += add;
        ws_items += w_new - w_old;
        ws_fixed = fixed;
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
    // a batch whose workspace does not fit in the free device memory is split: the later
    // half of its requests goes back to the front of the queue (arrival order kept) and the
    // first half is launched, down to a single request
    while (st == TDA_ENOMEM && take.size() > 1) {
      const size_t half = take.size() / 2;
      lk.lock();
      for (size_t i = take.size(); i-- > half;) pending.push_front(take[i]);
      lk.unlock();
      take.resize(half);
      st = launch(sl, take, dsv);
    }
    lk.lock();
    if (st != TDA_OK) {
      error = st;
      error_msg = tda_last_error();
      for (const Request &r : take) finish(r.ticket, 2);
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
      finish(r.ticket, e == hipSuccess ? 1 : 2);
      lat.add((t - r.t_submit) * 1e3);
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
  // a launch gathers at most slot_rows templates (a single request may fill the share)
  const size_t slot_rows = s->slot_stage_bytes / (sizeof(void *) + sizeof(double));
  // outstanding requests: at most max_queue pending plus what n_slots launches took
  const uint64_t most = (uint64_t)opt->max_queue * (uint64_t)(opt->n_slots + 1);
  uint64_t rs = 1024;
  while (rs < 2 * most) rs <<= 1;
  if (rs > ((uint64_t)1 << 30)) {
    delete s;
    return set_error(TDA_EINVAL, "max_queue x (n_slots + 1) too large for the request ring");
  }
  s->ring.assign(rs, 0);
  s->ring_mask = rs - 1;
  s->max_outstanding = (int64_t)most;
  s->slots.resize(opt->n_slots);
  for (Slot &sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      delete s;
      return set_error(TDA_EHIP, "server: stream/event creation failed");
    }
    sl.mc = multi_ctx_create();
    sl.rows_cap = slot_rows;
    sl.desc_cap = slot_rows;
    if (hipMalloc(&sl.rows_dev, slot_rows * sizeof(void *)) != hipSuccess ||
        hipMalloc((void **)&sl.out_dev, slot_rows * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&sl.desc_dev, slot_rows * 3 * sizeof(int64_t)) != hipSuccess ||
        hipHostMalloc(&sl.rows_host, slot_rows * sizeof(void *), 0) != hipSuccess ||
        hipHostMalloc((void **)&sl.desc_host, slot_rows * 3 * sizeof(int64_t), 0) != hipSuccess) {
      tda_server_destroy(s);
      return set_error(TDA_ENOMEM, "server: slot table allocation failed");
    }
  }
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
  // one handle caches one data vector: a second registration with other data would
  // rewrite the cache under requests of the first
  for (size_t k = 0; k < s->ds.size(); ++k)
    if (s->ds[k].h == h) {
      if (s->ds[k].d != d)
        return set_error(TDA_EINVAL, "handle already registered with other data");
      *dataset = (int32_t)k;
      return TDA_OK;
    }
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
  if ((int64_t)s->pending.size() >= s->opt.max_queue || s->outstanding >= s->max_outstanding ||
      (size_t)B * (sizeof(void *) + sizeof(double)) > s->slot_stage_bytes) {
    s->rejected += 1;
    return TDA_EAGAIN;
  }
  const uint64_t tk = s->next_ticket++;
  s->state(tk) = 0;
  s->outstanding += 1;
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
  const uint8_t st = s->status(ticket);
  if (st == 2) return set_error(TDA_EHIP, ("request failed: " + s->error_msg).c_str());
  *done = st == 1;
  return TDA_OK;
}

extern "C" tda_status tda_server_wait(tda_server_t s, uint64_t ticket, double timeout_s) {
  if (!s) return set_error(TDA_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return set_error(TDA_EINVAL, "unknown ticket");
  const bool ok = s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                 [&] { return s->status(ticket) != 0; });
  if (!ok) return TDA_EAGAIN;
  return s->status(ticket) == 1 ? TDA_OK
                                 : set_error(TDA_EHIP, ("request failed: " + s->error_msg).c_str());
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
  if (s->lat.count) {
    st->p50_ms = s->lat.pct(50);
    st->p99_ms = s->lat.pct(99);
    st->mean_ms = s->lat.sum / (double)s->lat.count;
    st->max_ms = s->lat.max;
  }
  st->mean_templates_per_launch = s->launches ? (double)s->templates / (double)s->launches : 0;
  if (reset) {
    s->lat.clear();
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
