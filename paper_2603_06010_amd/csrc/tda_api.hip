// libtda C ABI: handles, device memory, validation and the launch sequences of the
// factorisation and of the FP64 / mixed-precision log-likelihood evaluations.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "tda_internal.h"

using namespace tda;

// Scratch of the allocation-free FP64 evaluation (tda_loglik_fp64_noalloc): the solution
// rows of its column tiles.  A fixed device array; every GPU the library runs on holds its
// own copy until the process ends.  Host code takes its per-device address from
// hipGetSymbolAddress and never uses the array's name as an address.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
namespace noalloc {
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];
}

namespace {

thread_local std::string g_err;

tda_status fail_with(tda_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

std::mutex g_noalloc_mu;
constexpr int kMaxDevices = 64;
double *g_noalloc_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array; the device must be current.
// hipGetSymbolAddress runs once per device (at the first tda_cov_build on it).
tda_status noalloc_scratch(int dev, double **out) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (dev < 0 || dev >= kMaxDevices) return fail_with(TDA_EINVAL, "device %d out of range", dev);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc::scratch));
    if (e != hipSuccess || !p)
      return fail_with(TDA_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_noalloc_ptr[dev] = (double *)p;
  }
  *out = g_noalloc_ptr[dev];
  return TDA_OK;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail_with(TDA_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                       __FILE__, __LINE__);                                                 \
  } while (0)

#define TDA_TRY(expr)            \
  do {                           \
    tda_status s_ = (expr);      \
    if (s_ != TDA_OK) return s_; \
  } while (0)

const double kLog2Pi = 1.8378770664093454835606594728112;

struct Seg {
  int64_t offset, length, n_keep, n_pad, row0;
  int32_t blk0, nblk;
  int64_t m;
  int32_t log2m;
};

// Device buffer with budget accounting.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Ring of pinned host staging slots and matching device buffers for per-call
// descriptors.  A slot is reused only after the work that read it has finished.
// Slot K is the graph slot: sized before a capture, used only while capturing (no
// waits or allocations there), and never recycled, because the captured graph copies
// from it on every replay.
struct DescRing {
  static constexpr int K = 4;
  void *host[K + 1] = {};
  void *dev[K + 1] = {};
  size_t cap[K + 1] = {};
  hipEvent_t ev[K] = {};
  int next = 0;
  int cur = -1;
  bool graph = false;     // calls go to the graph slot
  size_t last_used = 0;   // bytes used by the last sealed call

  hipError_t grow(int slot, size_t need) {
    if (host[slot]) hipHostFree(host[slot]);
    if (dev[slot]) hipFree(dev[slot]);
    host[slot] = dev[slot] = nullptr;
    cap[slot] = 0;
    const size_t c = std::max(need * 2, (size_t)1 << 16);
    hipError_t e = hipHostMalloc(&host[slot], c, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = hipMalloc(&dev[slot], c);
    if (e != hipSuccess) return e;
    cap[slot] = c;
    return hipSuccess;
  }
  // Size the graph slot (outside any capture) and route the next calls to it.
  hipError_t begin_graph(size_t need) {
    if (need > cap[K]) {
      hipError_t e = grow(K, need);
      if (e != hipSuccess) return e;
    }
    graph = true;
    cur = -1;
    return hipSuccess;
  }
  void end_graph() {
    graph = false;
    cur = -1;
  }
  // Returns a device pointer holding a copy of `data` (enqueued on s).
  hipError_t push(const void *data, size_t n, hipStream_t s, void **dptr) {
    if (cur < 0) {
      if (graph) {
        cur = K;
      } else {
        cur = next;
        next = (next + 1) % K;
        if (ev[cur]) {
          hipError_t e = hipEventSynchronize(ev[cur]);
          if (e != hipSuccess) return e;
        }
      }
      used = 0;
    }
    const size_t need = used + ((n + 255) & ~(size_t)255);
    if (need > cap[cur]) {
      // one growth per call, before any push; never while capturing
      if (used || cur == K) return hipErrorInvalidValue;
      hipError_t e = grow(cur, need);
      if (e != hipSuccess) return e;
    }
    memcpy((char *)host[cur] + used, data, n);
    hipError_t e = hipMemcpyAsync((char *)dev[cur] + used, (char *)host[cur] + used, n,
                                  hipMemcpyHostToDevice, s);
    *dptr = (char *)dev[cur] + used;
    used = need;
    return e;
  }
  // Reserve room for a whole call up front (so a call never grows mid-way).
  hipError_t reserve(size_t total) {
    if (cur >= 0) return hipSuccess;
    if (graph) {
      if (total > cap[K]) return hipErrorInvalidValue;
      cur = K;
      used = 0;
      return hipSuccess;
    }
    int slot = next;
    if (ev[slot]) {
      hipError_t e = hipEventSynchronize(ev[slot]);
      if (e != hipSuccess) return e;
    }
    if (total > cap[slot]) {
      hipError_t e = grow(slot, total);
      if (e != hipSuccess) return e;
    }
    cur = slot;
    next = (next + 1) % K;
    used = 0;
    return hipSuccess;
  }
  hipError_t seal(hipStream_t s) {
    if (cur < 0) return hipSuccess;
    last_used = used;
    if (cur == K) {  // graph slot: nothing to wait for later
      cur = -1;
      return hipSuccess;
    }
    if (!ev[cur]) {
      hipError_t e = hipEventCreateWithFlags(&ev[cur], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(ev[cur], s);
    cur = -1;
    return e;
  }
  void destroy() {
    for (int k = 0; k <= K; ++k) {
      if (k < K && ev[k]) hipEventSynchronize(ev[k]), hipEventDestroy(ev[k]);
      if (host[k]) hipHostFree(host[k]);
      if (dev[k]) hipFree(dev[k]);
      host[k] = dev[k] = nullptr;
      if (k < K) ev[k] = nullptr;
      cap[k] = 0;
    }
  }
  size_t used = 0;
};

}  // namespace

struct tda_ctx {
  int device = 0;
  tda_allocator user_alloc{};  // caller's device-memory provider (has_user_alloc)
  bool has_user_alloc = false;
  int precision = TDA_PREC_FP64;
  int flags = 0;
  bool compacted = false;  // FP64 panels and operator released (TDA_FLAG_COMPACT)
  size_t budget = 0;
  size_t held = 0;
  int64_t N = 0, n_eff = 0, n_pad = 0;
  int32_t nblk = 0;
  std::vector<Seg> segs;
  std::vector<double> acf;
  std::vector<int32_t> blk_first_h, blk_last_h;
  std::vector<int64_t> panel_off_h;
  int64_t panel_total = 0;

  // device state
  DevBuf acf_d, idx_d, pos2row_d, blk_first_d, blk_last_d;
  DevBuf retpos_d;     // [n_pad] position of each padded row among the retained samples, -1 = padding
  std::vector<int32_t> idx_h;  // host copy of idx (sample of each padded row, -1 = padding)
  uint64_t idx_hash = 0;       // FNV-1a of idx_h
  DevBuf A_d;          // dense per-segment blocks (until factored)
  DevBuf dinv128_d, dinv256_d, logdiag_d, logdet_d, fail_d;
  DevBuf panels_d, panel_off_d;
  double logdet = 0.0;
  bool factored = false;
  int64_t fail_row = -1;
  int32_t fail_segment = -1;

  // mixed state
  DevBuf w64_d, w64_off_d, w64_rb_d;
  DevBuf wa_hi, wa_lo, wb_hi, wb_lo, wa_off_d, wb_off_d;
  DevBuf lam_d, tw_d, segdev_d;
  DevBuf dbar_d, yd_d, ydpos_d;
  DevBuf cache_d;   // DataCache: fingerprint and q_dd of the whitened data
  DevBuf chk_d;     // DataCheck of the single-handle calls (serialised per handle)
  const double *data_ptr = nullptr;  // data of the last call (compact handles: the cached data)

  // Gohberg-Semencul state: per segment twiddles, pass twiddles, the two spectra and
  // x = C^-1 e_1; descriptors; Levinson outputs
  DevBuf gs_tab_d, gs_seg_d, gs_lev_d;
  std::vector<GsSeg> gs_seg_h;
  int64_t gs_max_len = 0;

  // workspaces
  DevBuf ws_scratch, ws_tiles, ws_items;
  DevBuf ws_hs_hi, ws_hs_lo, ws_w0_hi, ws_w0_lo, ws_y0, ws_fft, ws_work, ws_mix, ws_ref;
  DevBuf ws_zero, ws_terms;  // inner-product entry point: zero vector [N], <h,h> and <d,d>
  DevBuf ws_cdo;             // explicit-inverse evaluation: residual rows and block sums
  DevBuf ws_snr;             // tda_snr: <d,h> and <h,h>
  hipEvent_t done = nullptr;  // last enqueued work of this handle
  DescRing ring;
  std::vector<SegDev> segdev_h;
  int64_t max_m = 0;
  std::vector<int64_t> w64_off_h;
  std::vector<int32_t> w64_rb_h;
  std::vector<int64_t> wa_off_h, wb_off_h;
  int64_t work_Bp = -1;      // Bp the cached mixed work lists were built for
  int64_t n_work_fwd = 0, n_work_bwd = 0;

  tda_status alloc(DevBuf &b, size_t bytes) {
    if (b.p) {
      if (b.bytes >= bytes) return TDA_OK;
      hipDeviceSynchronize();
      free_dev(b.p);
      held -= b.bytes;
      b.p = nullptr;
      b.bytes = 0;
    }
    // whole 512-byte units (the granule of PyTorch's caching allocator, so that the bytes a
    // caller's allocator accounts equal device_bytes)
    if (bytes == 0) bytes = 512;
    bytes = (bytes + 511) & ~(size_t)511;
    if (budget && held + bytes > budget)
      return fail_with(TDA_ENOMEM, "HBM budget exceeded: need %zu more bytes, hold %zu of %zu",
                       bytes, held, budget);
    if (has_user_alloc) {
      b.p = user_alloc.alloc(bytes, user_alloc.ctx);
      if (!b.p) {
        (void)hipGetLastError();  // a failed device allocation inside the allocator, as above
        return fail_with(TDA_ENOMEM, "allocator returned NULL for %zu bytes", bytes);
      }
      if ((uintptr_t)b.p & 255) {
        user_alloc.free(b.p, user_alloc.ctx);
        b.p = nullptr;
        return fail_with(TDA_ENOMEM, "allocator returned memory not aligned to 256 bytes");
      }
    } else {
      hipError_t e = hipMalloc(&b.p, bytes);
      if (e != hipSuccess) {
        b.p = nullptr;
        // the runtime also records the failure as the thread's last error; clear it, or the
        // next kernel launch check would report it as its own
        (void)hipGetLastError();
        return fail_with(TDA_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
      }
    }
    b.bytes = bytes;
    held += bytes;
    return TDA_OK;
  }
  void free_dev(void *p) {
    if (has_user_alloc)
      user_alloc.free(p, user_alloc.ctx);
    else
      hipFree(p);
  }
  void release(DevBuf &b) {
    if (b.p) {
      free_dev(b.p);
      held -= b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
  }
  void release_all() {
    DevBuf *all[] = {&acf_d,   &idx_d,    &pos2row_d,  &blk_first_d, &blk_last_d, &A_d,
                     &dinv128_d, &dinv256_d, &logdiag_d, &logdet_d,  &fail_d,     &panels_d,
                     &panel_off_d, &w64_d, &w64_off_d, &w64_rb_d,    &wa_hi,      &wa_lo,
                     &wb_hi,   &wb_lo,    &wa_off_d,   &wb_off_d,    &lam_d,      &tw_d,
                     &segdev_d, &dbar_d,  &yd_d,       &ydpos_d,     &cache_d,    &ws_scratch,
                     &ws_tiles, &ws_items, &ws_hs_hi,  &ws_hs_lo,    &ws_w0_hi,   &ws_w0_lo,
                     &ws_y0,   &ws_fft,   &ws_work,    &ws_mix,      &ws_ref,     &gs_tab_d,
                     &gs_seg_d, &gs_lev_d, &ws_zero,  &ws_terms,   &ws_cdo,      &retpos_d,
                     &chk_d,   &ws_snr};
    for (DevBuf *b : all) release(*b);
  }
  double cterm() const { return -0.5 * logdet - 0.5 * (double)n_eff * kLog2Pi; }
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    hipGetDevice(&prev);
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

std::once_flag g_attr_once;
void set_kernel_attributes();

tda_status upload(tda_ctx *h, DevBuf &b, const void *src, size_t bytes) {
  TDA_TRY(h->alloc(b, bytes));
  HIP_TRY(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
  return TDA_OK;
}

// Wait (on `s`) for the handle's previous work, so workspaces are never shared by two
// calls that run concurrently on different streams.
tda_status order_after_previous(tda_ctx *h, hipStream_t s) {
  if (!h->done) HIP_TRY(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
  HIP_TRY(hipStreamWaitEvent(s, h->done, 0));
  return TDA_OK;
}

tda_status mark_done(tda_ctx *h, hipStream_t s) {
  HIP_TRY(hipEventRecord(h->done, s));
  return TDA_OK;
}

}  // namespace

// ---------------------------------------------------------------- build

extern "C" tda_status tda_cov_build(const double *acf, int64_t acf_len, int64_t N,
                                    const uint8_t *gap_mask, const tda_segment *segments,
                                    int64_t n_segments, const tda_options *opt, tda_handle *out) {
  if (!out) return fail_with(TDA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!acf) return fail_with(TDA_EINVAL, "acf is NULL");
  if (N < 1) return fail_with(TDA_EINVAL, "N must be >= 1");
  if (N > (int64_t)1 << 30) return fail_with(TDA_EINVAL, "N too large");
  if (!(acf_len >= 1) || !(acf[0] > 0.0) || !isfinite(acf[0]))
    return fail_with(TDA_EINVAL, "acf[0] must be positive and finite");
  if (n_segments < 0 || (n_segments > 0 && !segments))
    return fail_with(TDA_EINVAL, "bad segment list");
  // struct_size, precision, device, flags, budget, allocator
  tda_options o{sizeof(tda_options), TDA_PREC_FP64, -1, 0, 0, nullptr};
  if (opt) {
    // the options of callers built before the allocator field end at its offset
    const size_t v1 = offsetof(tda_options, allocator);
    if (opt->struct_size < v1) return fail_with(TDA_EINVAL, "options struct_size");
    memcpy(&o, opt, std::min<size_t>(opt->struct_size, sizeof(tda_options)));
    o.struct_size = sizeof(tda_options);
  }
  if (o.allocator && (!o.allocator->alloc || !o.allocator->free))
    return fail_with(TDA_EINVAL, "allocator needs both alloc and free");
  if (o.precision != TDA_PREC_FP64 && o.precision != TDA_PREC_MIXED && o.precision != TDA_PREC_GS)
    return fail_with(TDA_EINVAL, "unknown precision %d", o.precision);
  if (o.flags & ~TDA_FLAG_COMPACT) return fail_with(TDA_EINVAL, "unknown flags");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail_with(TDA_ENODEV, "no HIP device");
  int dev = o.device;
  if (dev < 0) hipGetDevice(&dev);
  if (dev >= ndev) return fail_with(TDA_EINVAL, "device %d out of range", dev);

  std::vector<tda_segment> segs;
  if (n_segments == 0)
    segs.push_back({0, N});
  else
    segs.assign(segments, segments + n_segments);
  int64_t prev_end = 0, longest = 0;
  for (size_t i = 0; i < segs.size(); ++i) {
    const tda_segment &s = segs[i];
    if (s.length < 1 || s.offset < prev_end || s.offset + s.length > N)
      return fail_with(TDA_EINVAL, "segment %zu must be non-empty, sorted, disjoint, inside [0,N)",
                       i);
    prev_end = s.offset + s.length;
    longest = std::max(longest, s.length);
  }
  if (acf_len < longest)
    return fail_with(TDA_EINVAL, "acf_len %lld shorter than the longest segment %lld",
                     (long long)acf_len, (long long)longest);
  for (int64_t i = 0; i < longest; ++i)
    if (!isfinite(acf[i])) return fail_with(TDA_EINVAL, "acf[%lld] is not finite", (long long)i);

  std::call_once(g_attr_once, set_kernel_attributes);
  DeviceGuard guard(dev);
  tda_ctx *h = new tda_ctx();
  h->device = dev;
  h->precision = o.precision;
  h->flags = o.flags;
  h->budget = o.hbm_budget_bytes;
  if (o.allocator) {
    h->user_alloc = *o.allocator;
    h->has_user_alloc = true;
  }
  h->N = N;
  h->acf.assign(acf, acf + longest);

  std::vector<int32_t> idx, pos2row((size_t)N, -1), retpos;
  int64_t row = 0;
  int32_t blk = 0;
  for (const tda_segment &s : segs) {
    Seg g{};
    g.offset = s.offset;
    g.length = s.length;
    g.row0 = row;
    g.blk0 = blk;
    int64_t keep = 0;
    for (int64_t j = s.offset; j < s.offset + s.length; ++j) {
      if (gap_mask && gap_mask[j]) continue;
      pos2row[j] = (int32_t)(row + keep);
      idx.push_back((int32_t)j);
      retpos.push_back((int32_t)(h->n_eff + keep));
      ++keep;
    }
    if (keep == 0) continue;  // a fully excluded segment contributes nothing
    g.n_keep = keep;
    g.n_pad = (keep + TB - 1) / TB * TB;
    for (int64_t j = keep; j < g.n_pad; ++j) {
      idx.push_back(-1);
      retpos.push_back(-1);
    }
    g.nblk = (int32_t)(g.n_pad / TB);
    int32_t l2 = 4;  // m >= 16: the in-LDS refinement needs m/4 >= 4
    while (((int64_t)1 << l2) < 2 * g.length) ++l2;
    g.log2m = l2;
    g.m = (int64_t)1 << l2;
    for (int32_t b = 0; b < g.nblk; ++b) {
      h->blk_first_h.push_back(g.blk0);
      h->blk_last_h.push_back(g.blk0 + g.nblk - 1);
    }
    row += g.n_pad;
    blk += g.nblk;
    h->n_eff += keep;
    h->segs.push_back(g);
  }
  if (h->n_eff == 0) {
    delete h;
    return fail_with(TDA_EINVAL, "no retained sample");
  }
  h->n_pad = row;
  h->nblk = blk;
  h->idx_h = idx;
  if (hipEventCreateWithFlags(&h->done, hipEventDisableTiming) != hipSuccess) {
    delete h;
    return fail_with(TDA_EHIP, "event creation failed");
  }
  {
    double *unused = nullptr;
    const tda_status st0 = noalloc_scratch(dev, &unused);
    if (st0 != TDA_OK) {
      hipEventDestroy(h->done);
      delete h;
      return st0;
    }
  }
  h->idx_hash = 1469598103934665603ull;
  for (int32_t v : idx) h->idx_hash = (h->idx_hash ^ (uint32_t)v) * 1099511628211ull;
  if (h->n_pad > ((int64_t)1 << 31) / TB) {
    hipEventDestroy(h->done);
    delete h;
    return fail_with(TDA_EINVAL, "too many rows");
  }
  // panel offsets: block row i of its segment has (local i + 1) * TB * TB doubles
  h->panel_off_h.resize(h->nblk);
  int64_t off = 0;
  for (const Seg &g : h->segs)
    for (int32_t i = 0; i < g.nblk; ++i) {
      h->panel_off_h[g.blk0 + i] = off;
      off += (int64_t)(i + 1) * TB * TB;
    }
  h->panel_total = off;

  tda_status st = TDA_OK;
  auto cleanup = [&](tda_status s) {
    h->release_all();
    hipEventDestroy(h->done);
    delete h;
    return s;
  };
  if ((st = upload(h, h->acf_d, h->acf.data(), h->acf.size() * sizeof(double))) != TDA_OK ||
      (st = upload(h, h->idx_d, idx.data(), idx.size() * sizeof(int32_t))) != TDA_OK ||
      (st = upload(h, h->pos2row_d, pos2row.data(), pos2row.size() * sizeof(int32_t))) != TDA_OK ||
      (st = upload(h, h->retpos_d, retpos.data(), retpos.size() * sizeof(int32_t))) != TDA_OK ||
      (st = upload(h, h->blk_first_d, h->blk_first_h.data(), h->nblk * sizeof(int32_t))) != TDA_OK ||
      (st = upload(h, h->blk_last_d, h->blk_last_h.data(), h->nblk * sizeof(int32_t))) != TDA_OK ||
      (st = upload(h, h->panel_off_d, h->panel_off_h.data(), h->nblk * sizeof(int64_t))) != TDA_OK)
    return cleanup(st);
  if (h->precision == TDA_PREC_GS) {
    // Gohberg-Semencul needs each segment Toeplitz (no excluded sample inside it)
    for (size_t si = 0; si < h->segs.size(); ++si) {
      const Seg &g = h->segs[si];
      if (g.n_keep != g.length)
        return cleanup(fail_with(TDA_EINVAL, "GS precision: segment %zu has excluded samples", si));
      if (g.length > GS_MAX_LEN)
        return cleanup(fail_with(TDA_EINVAL, "GS precision: segment %zu is longer than %d samples",
                                 si, GS_MAX_LEN));
    }
  } else {
    // dense blocks (lower triangle used), assembled now
    size_t dense = 0;
    for (const Seg &g : h->segs) dense += (size_t)g.n_pad * g.n_pad;
    if ((st = h->alloc(h->A_d, dense * sizeof(double))) != TDA_OK) return cleanup(st);
    size_t a_off = 0;
    for (const Seg &g : h->segs) {
      TimedScope ts("assemble", 0);
      hipError_t e = launch_assemble((const double *)h->acf_d.p,
                                     (const int32_t *)h->idx_d.p + g.row0, g.n_keep, g.n_pad,
                                     (double *)h->A_d.p + a_off, 0);
      if (e != hipSuccess)
        return cleanup(fail_with(TDA_EHIP, "assemble launch: %s", hipGetErrorString(e)));
      a_off += (size_t)g.n_pad * g.n_pad;
    }
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return cleanup(fail_with(TDA_EHIP, "assemble: %s", hipGetErrorString(e)));
  *out = h;
  return TDA_OK;
}

// ---------------------------------------------------------------- factor

static tda_status build_mixed(tda_ctx *h);
static tda_status build_gs(tda_ctx *h);

extern "C" tda_status tda_factor(tda_handle h) {
  if (!h) return fail_with(TDA_EINVAL, "NULL handle");
  if (h->factored) return TDA_OK;
  if (h->precision == TDA_PREC_GS) {
    DeviceGuard guard(h->device);
    TDA_TRY(build_gs(h));
    h->factored = true;
    return TDA_OK;
  }
  if (!h->A_d.p) return fail_with(TDA_ESTATE, "handle has no assembled covariance");
  DeviceGuard guard(h->device);
  int64_t ncp = 0;
  for (const Seg &g : h->segs) ncp += g.n_pad / CP;
  TDA_TRY(h->alloc(h->dinv128_d, (size_t)ncp * CP * CP * sizeof(double)));
  TDA_TRY(h->alloc(h->dinv256_d, (size_t)h->nblk * TB * TB * sizeof(double)));
  TDA_TRY(h->alloc(h->logdiag_d, (size_t)ncp * sizeof(double)));
  TDA_TRY(h->alloc(h->logdet_d, sizeof(double)));
  TDA_TRY(h->alloc(h->fail_d, sizeof(int32_t)));
  TDA_TRY(h->alloc(h->panels_d, (size_t)h->panel_total * sizeof(double)));
  size_t a_off = 0;
  int64_t cp_off = 0;
  for (size_t si = 0; si < h->segs.size(); ++si) {
    const Seg &g = h->segs[si];
    int32_t minus1 = -1;
    HIP_TRY(hipMemcpy(h->fail_d.p, &minus1, sizeof minus1, hipMemcpyHostToDevice));
    double *A = (double *)h->A_d.p + a_off;
    double *dinv = (double *)h->dinv128_d.p + cp_off * CP * CP;
    {
      TimedScope ts("cholesky", 0);
      HIP_TRY(launch_cholesky(A, g.n_pad, dinv, (double *)h->logdiag_d.p + cp_off,
                              (int32_t *)h->fail_d.p, 0));
    }
    int32_t failrow = -1;
    HIP_TRY(hipMemcpy(&failrow, h->fail_d.p, sizeof failrow, hipMemcpyDeviceToHost));
    if (failrow >= 0) {
      h->fail_row = failrow;
      h->fail_segment = (int32_t)si;
      return fail_with(TDA_ENOTSPD,
                       "covariance not positive definite: pivot of retained row %d of segment %zu",
                       failrow, si);
    }
    double *d256 = (double *)h->dinv256_d.p + (int64_t)g.blk0 * TB * TB;
    HIP_TRY(launch_diag_inverse(A, g.n_pad, dinv, d256, 0));
    HIP_TRY(launch_pack_panels(A, g.n_pad, g.row0, d256, (double *)h->panels_d.p,
                               (const int64_t *)h->panel_off_d.p, g.blk0, g.nblk, 0));
    a_off += (size_t)g.n_pad * g.n_pad;
    cp_off += g.n_pad / CP;
  }
  HIP_TRY(launch_sum_logdet((const double *)h->logdiag_d.p, ncp, (double *)h->logdet_d.p, 0));
  HIP_TRY(hipMemcpy(&h->logdet, h->logdet_d.p, sizeof(double), hipMemcpyDeviceToHost));
  h->release(h->A_d);
  h->release(h->dinv128_d);
  h->release(h->dinv256_d);
  if (!isfinite(h->logdet)) return fail_with(TDA_ENOTSPD, "log det is not finite");
  if (h->precision == TDA_PREC_MIXED) TDA_TRY(build_mixed(h));
  h->factored = true;
  return TDA_OK;
}

// ---------------------------------------------------------------- Gohberg-Semencul set-up

// Per segment (tables in doubles): twiddles w_m^r (2m), pass twiddles (2 m/4), the two
// correlation spectra (2m each) and x = C^-1 e_1 (length).
static tda_status build_gs(tda_ctx *h) {
  const size_t ns = h->segs.size();
  std::vector<size_t> base(ns);
  size_t tot = 0;
  for (size_t si = 0; si < ns; ++si) {
    const Seg &g = h->segs[si];
    base[si] = tot;
    tot += (size_t)(2 * g.m + 2 * (g.m / 4) + 4 * g.m + g.length);
  }
  TDA_TRY(h->alloc(h->gs_tab_d, tot * sizeof(double)));
  TDA_TRY(h->alloc(h->gs_lev_d, ns * (sizeof(double) + sizeof(int32_t))));
  double *tab = (double *)h->gs_tab_d.p;
  double *ld_d = (double *)h->gs_lev_d.p;
  int32_t *fail_d = (int32_t *)(ld_d + ns);
  for (size_t si = 0; si < ns; ++si) {
    const Seg &g = h->segs[si];
    double *tw = tab + base[si], *ptw = tw + 2 * g.m, *M1 = ptw + 2 * (g.m / 4), *M2 = M1 + 2 * g.m;
    double *x = M2 + 2 * g.m;
    HIP_TRY(launch_lambda((const double *)h->acf_d.p, g.length, g.m, tw, nullptr, ptw, 0));
    HIP_TRY(launch_levinson((const double *)h->acf_d.p, g.length, x, ld_d + si, fail_d + si, 0));
    HIP_TRY(launch_gs_spectra(x, g.length, g.m, tw, M1, M2, 0));
  }
  HIP_TRY(hipDeviceSynchronize());
  std::vector<double> ld(ns);
  std::vector<int32_t> fail(ns);
  HIP_TRY(hipMemcpy(ld.data(), ld_d, ns * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(fail.data(), fail_d, ns * sizeof(int32_t), hipMemcpyDeviceToHost));
  h->gs_seg_h.clear();
  h->logdet = 0.0;
  h->gs_max_len = 0;
  h->max_m = 0;
  for (size_t si = 0; si < ns; ++si) {
    const Seg &g = h->segs[si];
    if (fail[si] >= 0) {
      h->fail_row = fail[si];
      h->fail_segment = (int32_t)si;
      return fail_with(TDA_ENOTSPD,
                       "covariance not positive definite: Levinson order %d of segment %zu",
                       fail[si], si);
    }
    double *tw = tab + base[si], *ptw = tw + 2 * g.m, *M1 = ptw + 2 * (g.m / 4), *M2 = M1 + 2 * g.m;
    double x0 = 0.0;
    HIP_TRY(hipMemcpy(&x0, M2 + 2 * g.m, sizeof(double), hipMemcpyDeviceToHost));
    if (!(x0 > 0.0) || !isfinite(x0)) return fail_with(TDA_ENOTSPD, "segment %zu: (C^-1)_00 = %g", si, x0);
    GsSeg sd{};
    sd.offset = g.offset;
    sd.length = g.length;
    sd.m = g.m;
    sd.log2m = g.log2m;
    sd.inv_x0 = 1.0 / x0;
    sd.tw = tw;
    sd.ptw = ptw;
    sd.M1 = M1;
    sd.M2 = M2;
    h->gs_seg_h.push_back(sd);
    h->logdet += ld[si];
    h->gs_max_len = std::max(h->gs_max_len, g.length);
    h->max_m = std::max(h->max_m, g.m);
  }
  if (!isfinite(h->logdet)) return fail_with(TDA_ENOTSPD, "log det is not finite");
  TDA_TRY(upload(h, h->gs_seg_d, h->gs_seg_h.data(), ns * sizeof(GsSeg)));
  return TDA_OK;
}

// Per-template transform work (in-LDS refinement, Gohberg-Semencul) in XCD order.
// Workgroup i of a launch runs on XCD i mod 8 and the persistent grid (a multiple of 8
// workgroups) keeps each workgroup's entries on it, so entry 8 q + x runs on XCD x.  The templates of one 32-template tile of the split layout go
// to one XCD, so the partial lines of the residual they write meet in that XCD's L2; tiles
// are dealt to the XCDs in turn, and each XCD's list is padded to the longest with empty
// entries (item -1).
static std::vector<int2> xcd_tiles(const std::vector<int2> &w) {
  constexpr int NX = 8;
  std::vector<std::vector<int2>> lists(NX);
  int j = 0;
  for (size_t n = 0; n < w.size();) {
    size_t e = n + 1;
    while (e < w.size() && w[e].x == w[n].x && w[e].y / 32 == w[n].y / 32) ++e;
    std::vector<int2> &l = lists[j++ % NX];
    l.insert(l.end(), w.begin() + n, w.begin() + e);
    n = e;
  }
  size_t len = 0;
  for (const auto &l : lists) len = std::max(len, l.size());
  std::vector<int2> out(len * NX, int2{-1, -1});
  for (int x = 0; x < NX; ++x)
    for (size_t q = 0; q < lists[x].size(); ++q) out[q * NX + x] = lists[x][q];
  return out;
}

constexpr int32_t kGsWG = 1024;  // persistent Gohberg-Semencul workgroups (one per CU runs at once)

// Per-workgroup Gohberg-Semencul scratch: the parked even parts of the two products (max_len
// doubles each, rounded to an even count) and, when a segment's transforms split in
// quarters, their quarters; fewer workgroups then.
struct GsScratch {
  int32_t n_wg;
  int64_t stride, qoff;
  size_t bytes;
};
static GsScratch gs_scratch_plan(int64_t n_work, int64_t max_len, int64_t max_m) {
  const bool quad = max_m > RL_MAX_M_SPLIT;
  GsScratch g;
  g.n_wg = (int32_t)std::min<int64_t>(n_work, quad ? RL_QUAD_WG : kGsWG);
  const int64_t tes = (max_len + 1) & ~(int64_t)1;
  g.qoff = quad ? 2 * tes : -1;
  g.stride = 2 * tes + (quad ? 2 * RL_QUAD_SCRATCH : 0);
  g.bytes = (size_t)g.n_wg * g.stride * sizeof(double);
  return g;
}

static GsItem make_gs_item(const tda_ctx *h, const double *d, const double *H, int64_t ldh,
                           int64_t B, double *out) {
  GsItem it{};
  it.segs = (const GsSeg *)h->gs_seg_d.p;
  it.n_segs = (int32_t)h->gs_seg_h.size();
  it.B = (int32_t)B;
  it.d = d;
  it.H = H;
  it.ldh = ldh;
  it.out = out;
  it.cterm = h->cterm();
  return it;
}

static tda_status loglik_gs(tda_ctx *h, const double *d, const double *H, int64_t B, int64_t ldh,
                            double *out, hipStream_t s) {
  std::vector<int2> work((size_t)B);
  for (int64_t b = 0; b < B; ++b) work[b] = int2{0, (int32_t)b};
  work = xcd_tiles(work);
  const GsScratch gsc = gs_scratch_plan((int64_t)work.size(), h->gs_max_len, h->max_m);
  TDA_TRY(h->alloc(h->ws_fft, gsc.bytes));
  const GsItem it = make_gs_item(h, d, H, ldh, B, out);
  HIP_TRY(h->ring.reserve(1024 + sizeof(GsItem) + work.size() * sizeof(int2)));
  void *d_it, *d_w;
  HIP_TRY(h->ring.push(&it, sizeof(GsItem), s, &d_it));
  HIP_TRY(h->ring.push(work.data(), work.size() * sizeof(int2), s, &d_w));
  {
    TimedScope ts("gs_fft", s);
    HIP_TRY(launch_gs((const GsItem *)d_it, (const int2 *)d_w, (int64_t)work.size(),
                      (double *)h->ws_fft.p, gsc.stride, gsc.qoff, gsc.n_wg, s));
  }
  HIP_TRY(h->ring.seal(s));
  return TDA_OK;
}

// ---------------------------------------------------------------- FP64 evaluation

static tda_status loglik_f64(tda_ctx *h, const double *d, const double *H, int64_t B, int64_t ldh,
                             double *out, hipStream_t s) {
  const int64_t ntile = (B + BC - 1) / BC;
  TDA_TRY(h->alloc(h->ws_scratch, (size_t)ntile * h->n_pad * BC * sizeof(double)));
  TrsmItem it{};
  it.panels = (const double *)h->panels_d.p;
  it.panel_off = (const int64_t *)h->panel_off_d.p;
  it.blk_first = (const int32_t *)h->blk_first_d.p;
  it.idx = (const int32_t *)h->idx_d.p;
  it.d = d;
  it.H = H;
  it.ldh = ldh;
  it.out = out;
  it.scratch = (double *)h->ws_scratch.p;
  it.cterm = h->cterm();
  it.B = (int32_t)B;
  it.mode = MODE_LOGLIK;
  {
    TimedScope ts("trsm_f64", s);
    HIP_TRY(launch_trsm_f64_single(it, h->nblk, ntile, s));
  }
  return TDA_OK;
}

static tda_status loglik_mixed(tda_ctx *h, const double *d, const double *H, int64_t B,
                               int64_t ldh, double *out, hipStream_t s, double *out_dh = nullptr,
                               double *out_hh = nullptr);
static tda_status loglik_cdo(tda_ctx *h, const double *d, const double *H, int64_t B,
                             int64_t ldh, double *out, hipStream_t s);

// Argument checks shared by the single-handle evaluation entry points.
static tda_status check_eval(tda_handle h, const double *d, const double *H, int64_t B,
                             int64_t ldh, const double *out, int32_t precision) {
  if (!h) return fail_with(TDA_EINVAL, "NULL handle");
  if (!h->factored) return fail_with(TDA_ESTATE, "tda_loglik before a successful tda_factor");
  if (B < 0) return fail_with(TDA_EINVAL, "B < 0");
  if (B == 0) return TDA_OK;
  if (B > (int64_t)1 << 30) return fail_with(TDA_EINVAL, "B too large");
  if (!d || !H || !out) return fail_with(TDA_EINVAL, "NULL device pointer");
  if (ldh < h->N) return fail_with(TDA_EINVAL, "ldh < N");
  if (precision != TDA_PREC_FP64 && precision != TDA_PREC_MIXED && precision != TDA_PREC_GS &&
      precision != TDA_PREC_CDO)
    return fail_with(TDA_EINVAL, "unknown precision");
  if (precision == TDA_PREC_MIXED && h->precision != TDA_PREC_MIXED)
    return fail_with(TDA_ESTATE, "mixed evaluation needs a handle built with TDA_PREC_MIXED");
  if (precision == TDA_PREC_CDO && (h->precision != TDA_PREC_MIXED || h->compacted))
    return fail_with(TDA_ESTATE, "explicit-inverse evaluation needs a (non-compact) mixed handle");
  if ((precision == TDA_PREC_GS) != (h->precision == TDA_PREC_GS))
    return fail_with(TDA_ESTATE, "a GS handle evaluates only (and only it) in TDA_PREC_GS");
  if (h->compacted && (precision == TDA_PREC_FP64 || d != h->data_ptr))
    return fail_with(TDA_ESTATE, "compact handle: only mixed evaluation with its cached data");
  return TDA_OK;
}

static tda_status refuse_capture(hipStream_t s) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cap));
  if (cap != hipStreamCaptureStatusNone)
    return fail_with(TDA_ESTATE, "stream capture outside a plan: use tda_plan_execute");
  return TDA_OK;
}

extern "C" tda_status tda_loglik_ex(tda_handle h, const double *d, const double *H, int64_t B,
                                    int64_t ldh, double *out, int32_t precision,
                                    void *hip_stream) {
  TDA_TRY(check_eval(h, d, H, B, ldh, out, precision));
  if (B == 0) return TDA_OK;
  DeviceGuard guard(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  TDA_TRY(refuse_capture(s));
  TDA_TRY(order_after_previous(h, s));
  if (precision == TDA_PREC_FP64)
    TDA_TRY(loglik_f64(h, d, H, B, ldh, out, s));
  else if (precision == TDA_PREC_GS)
    TDA_TRY(loglik_gs(h, d, H, B, ldh, out, s));
  else if (precision == TDA_PREC_CDO)
    TDA_TRY(loglik_cdo(h, d, H, B, ldh, out, s));
  else
    TDA_TRY(loglik_mixed(h, d, H, B, ldh, out, s));
  return mark_done(h, s);
}

// logL, <d,h> and <h,h> (either may be NULL) on stream s, ordered after the handle's
// earlier work by the caller.
static tda_status terms_impl(tda_ctx *h, const double *d, const double *H, int64_t B, int64_t ldh,
                             double *out, double *out_dh, double *out_hh, int32_t precision,
                             hipStream_t s) {
  if (precision == TDA_PREC_MIXED) {
    // <d,h> = y_d^T h is an FP64 term of the split form and <h,h> its refined part plus
    // the correction: both come out of the same launches
    return loglik_mixed(h, d, H, B, ldh, out, s, out_dh, out_hh);
  }
  auto eval = [&](const double *dd, const double *HH, int64_t BB, int64_t ld, double *o) {
    return precision == TDA_PREC_FP64  ? loglik_f64(h, dd, HH, BB, ld, o, s)
           : precision == TDA_PREC_CDO ? loglik_cdo(h, dd, HH, BB, ld, o, s)
                                       : loglik_gs(h, dd, HH, BB, ld, o, s);
  };
  TDA_TRY(eval(d, H, B, ldh, out));
  if (out_dh || out_hh) {
    // the same evaluation against zero data gives <h,h>, and the data against a zero
    // template <d,d>; <d,h> follows from the three
    if (!h->ws_zero.p) {
      TDA_TRY(h->alloc(h->ws_zero, (size_t)h->N * sizeof(double)));
      HIP_TRY(hipMemsetAsync(h->ws_zero.p, 0, (size_t)h->N * sizeof(double), s));
    }
    TDA_TRY(h->alloc(h->ws_terms, (size_t)(B + 1) * sizeof(double)));
    const double *zero = (const double *)h->ws_zero.p;
    double *hh = out_hh ? out_hh : (double *)h->ws_terms.p + 1;
    double *dd = (double *)h->ws_terms.p;
    TDA_TRY(eval(zero, H, B, ldh, hh));
    if (out_dh) TDA_TRY(eval(d, zero, 1, h->N, dd));
    HIP_TRY(launch_terms_combine(out, hh, dd, h->cterm(), B, out_dh, s));
  }
  return TDA_OK;
}

extern "C" tda_status tda_loglik_terms(tda_handle h, const double *d, const double *H, int64_t B,
                                       int64_t ldh, double *out, double *out_dh, double *out_hh,
                                       int32_t precision, void *hip_stream) {
  TDA_TRY(check_eval(h, d, H, B, ldh, out, precision));
  if (B == 0) return TDA_OK;
  DeviceGuard guard(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  TDA_TRY(refuse_capture(s));
  TDA_TRY(order_after_previous(h, s));
  TDA_TRY(terms_impl(h, d, H, B, ldh, out, out_dh, out_hh, precision, s));
  return mark_done(h, s);
}

extern "C" tda_status tda_snr(tda_handle h, const double *d, const double *H, int64_t B,
                              int64_t ldh, double *out, double *rho_mf, double *rho_opt,
                              double *rho_eff2, int32_t precision, void *hip_stream) {
  TDA_TRY(check_eval(h, d, H, B, ldh, out, precision));
  if (B == 0) return TDA_OK;
  DeviceGuard guard(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  TDA_TRY(refuse_capture(s));
  TDA_TRY(order_after_previous(h, s));
  // <d,h> and <h,h> into the handle's SNR buffer, then the three ratios
  TDA_TRY(h->alloc(h->ws_snr, (size_t)2 * B * sizeof(double)));
  double *dh = (double *)h->ws_snr.p, *hh = dh + B;
  TDA_TRY(terms_impl(h, d, H, B, ldh, out, dh, hh, precision, s));
  HIP_TRY(launch_snr(dh, hh, B, rho_mf, rho_opt, rho_eff2, s));
  return mark_done(h, s);
}

extern "C" tda_status tda_whitened_residual(tda_handle h, const double *d, const double *H,
                                            int64_t B, int64_t ldh, double *out, double *wres,
                                            int64_t ldw, void *hip_stream) {
  TDA_TRY(check_eval(h, d, H, B, ldh, out, TDA_PREC_FP64));
  if (B == 0) return TDA_OK;
  if (!wres) return fail_with(TDA_EINVAL, "NULL device pointer");
  if (ldw < h->n_eff) return fail_with(TDA_EINVAL, "ldw < n_eff");
  if (!h->panels_d.p) return fail_with(TDA_ESTATE, "whitened residuals need the FP64 factor");
  DeviceGuard guard(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  TDA_TRY(refuse_capture(s));
  TDA_TRY(order_after_previous(h, s));
  // the triangular solve leaves every template's w = L^-1 (d - h) in its scratch rows
  TDA_TRY(loglik_f64(h, d, H, B, ldh, out, s));
  {
    TimedScope ts("whiten_export", s);
    HIP_TRY(launch_whiten_export((const double *)h->ws_scratch.p, (const int32_t *)h->retpos_d.p,
                                 h->n_pad, B, wres, ldw, s));
  }
  return mark_done(h, s);
}

extern "C" tda_status tda_loglik(tda_handle h, const double *d, const double *H, int64_t B,
                                 int64_t ldh, double *out, void *hip_stream) {
  if (!h) return fail_with(TDA_EINVAL, "NULL handle");
  return tda_loglik_ex(h, d, H, B, ldh, out, h->precision, hip_stream);
}

// ---------------------------------------------------------------- allocation-free FP64 evaluation

extern "C" tda_status tda_loglik_fp64_noalloc(tda_handle h, const double *d, const double *H,
                                              int64_t B, int64_t ldh, double *out,
                                              void *hip_stream) {
  TDA_TRY(check_eval(h, d, H, B, ldh, out, TDA_PREC_FP64));
  if (B == 0) return TDA_OK;
  if (!h->panels_d.p) return fail_with(TDA_ESTATE, "FP64 evaluation needs the FP64 factor");
  const int64_t ntile = (B + BC - 1) / BC;
  const size_t need = (size_t)ntile * h->n_pad * BC * sizeof(double);
  if (need > kNoAllocScratchBytes)
    return fail_with(TDA_EINVAL,
                     "allocation-free evaluation needs %zu bytes of scratch, more than its %zu: "
                     "at most %lld templates at this size",
                     need, kNoAllocScratchBytes,
                     (long long)(kNoAllocScratchBytes / (h->n_pad * BC * sizeof(double)) * BC));
  DeviceGuard guard(h->device);
  double *scr = nullptr;
  TDA_TRY(noalloc_scratch(h->device, &scr));
  hipStream_t s = (hipStream_t)hip_stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (!capturing) TDA_TRY(order_after_previous(h, s));
  TrsmItem it{};
  it.panels = (const double *)h->panels_d.p;
  it.panel_off = (const int64_t *)h->panel_off_d.p;
  it.blk_first = (const int32_t *)h->blk_first_d.p;
  it.idx = (const int32_t *)h->idx_d.p;
  it.d = d;
  it.H = H;
  it.ldh = ldh;
  it.out = out;
  it.scratch = scr;
  it.cterm = h->cterm();
  it.B = (int32_t)B;
  it.mode = MODE_LOGLIK;
  HIP_TRY(launch_trsm_f64_single(it, h->nblk, ntile, s));
  if (!capturing) TDA_TRY(mark_done(h, s));
  return TDA_OK;
}

// ---------------------------------------------------------------- mixed precision

namespace {

// A product job: one block pair of an item, with its template groups and halves.
struct BlockJob {
  int32_t item, block, ntg, nsub;
  int64_t k;  // work weight (K blocks the pair spans)
};

// Product work order.  Workgroup g runs on XCD g mod 8, and each XCD has its own L2, so
// the list is built per XCD and interleaved.  Work is cut into super-tiles of kRB
// consecutive block pairs of one item x kTG template groups, the workgroups an XCD runs
// at once (64 half-group or 32 full-group ones): they share each operator k-step among
// kTG groups and each template k-step among kRB pairs in L2.  Pairs of one segment span
// the same K and their K walks are aligned (see the product kernels), so a super-tile's
// workgroups start and finish together and stay on the same k-steps.  Super-tiles go to
// the XCD with the least work so far, longest first.
constexpr int kRB = 4, kTG = 8;
std::vector<int4> xcd_order(std::vector<BlockJob> jobs) {
  constexpr int NX = 8;
  struct Tile {
    int64_t work;
    std::vector<int4> wg;
  };
  std::vector<Tile> tiles;
  size_t n = 0;
  while (n < jobs.size()) {
    // a run of consecutive blocks of one item
    size_t e = n;
    while (e < jobs.size() && e - n < (size_t)kRB && jobs[e].item == jobs[n].item) ++e;
    const int32_t ntg = jobs[n].ntg, nsub = jobs[n].nsub;
    // fewer blocks in the run (end of an item): more groups, about 32 workgroups per tile
    const int32_t tg = std::min<int32_t>(ntg, std::max<int32_t>(kTG, 32 / (int32_t)(e - n)));
    for (int32_t t0 = 0; t0 < ntg; t0 += tg) {
      Tile T{0, {}};
      for (int32_t t = t0; t < std::min(ntg, t0 + tg); ++t)
        for (size_t q = n; q < e; ++q)
          for (int32_t u = 0; u < nsub; ++u) {
            T.wg.push_back(int4{jobs[q].item, jobs[q].block, t, u});
            T.work += jobs[q].k;
          }
      tiles.push_back(std::move(T));
    }
    n = e;
  }
  std::stable_sort(tiles.begin(), tiles.end(),
                   [](const Tile &x, const Tile &y) { return x.work > y.work; });
  std::vector<std::vector<int4>> lists(NX);
  int64_t load[NX] = {};
  for (Tile &T : tiles) {
    int x = 0;
    for (int c = 1; c < NX; ++c)
      if (load[c] < load[x]) x = c;
    load[x] += T.work;
    lists[x].insert(lists[x].end(), T.wg.begin(), T.wg.end());
  }
  size_t longest = 0;
  for (int x = 0; x < NX; ++x) longest = std::max(longest, lists[x].size());
  std::vector<int4> out(longest * NX, int4{0, -1, 0, 0});
  for (int x = 0; x < NX; ++x)
    for (size_t k = 0; k < lists[x].size(); ++k) out[k * NX + x] = lists[x][k];
  return out;
}

constexpr int kRefineWG = 768;  // persistent refinement workgroups (3 per CU)

// FFT scratch of a launch whose largest circulant is max_m: the global-scratch refinement
// (m beyond the quarter split) or the quarters of the in-LDS one; none below that.
static size_t fft_ws_bytes(int64_t max_m) {
  if (max_m > RL_MAX_M_QUAD) return (size_t)kRefineWG * max_m * 16;
  if (max_m > RL_MAX_M_SPLIT) return (size_t)RL_QUAD_WG * RL_QUAD_SCRATCH * 16;
  return 0;
}

}  // namespace

static tda_status build_mixed(tda_ctx *h) {
  for (const Seg &g : h->segs)
    if (g.m > ((int64_t)1 << 18))
      return fail_with(TDA_EINVAL, "mixed precision supports segments of at most 131072 samples");
  const int64_t nct = h->n_pad / 32;
  h->w64_off_h.resize(nct);
  h->w64_rb_h.resize(nct);
  std::vector<TrsmTile> tiles(nct);
  int64_t off = 0;
  for (int64_t ct = 0; ct < nct; ++ct) {
    const int32_t blk = (int32_t)(ct * 32 / TB);
    const int32_t last = h->blk_last_h[blk];
    h->w64_off_h[ct] = off;
    h->w64_rb_h[ct] = blk * TB;
    tiles[ct] = TrsmTile{0, (int32_t)(ct * 32), blk, last + 1, off};
    off += (int64_t)(last + 1 - blk) * TB * 32;
  }
  TDA_TRY(h->alloc(h->w64_d, (size_t)off * sizeof(double)));
  TDA_TRY(upload(h, h->w64_off_d, h->w64_off_h.data(), nct * sizeof(int64_t)));
  TDA_TRY(upload(h, h->w64_rb_d, h->w64_rb_h.data(), nct * sizeof(int32_t)));
  // W = L^-1 by the FP64 solve against identity columns (rows above a column are zero
  // and skipped).
  TrsmItem it{};
  it.panels = (const double *)h->panels_d.p;
  it.panel_off = (const int64_t *)h->panel_off_d.p;
  it.blk_first = (const int32_t *)h->blk_first_d.p;
  it.idx = (const int32_t *)h->idx_d.p;
  it.scratch = (double *)h->w64_d.p;
  it.B = (int32_t)h->n_pad;
  it.mode = MODE_IDENTITY;
  TDA_TRY(upload(h, h->ws_items, &it, sizeof it));
  TDA_TRY(upload(h, h->ws_tiles, tiles.data(), tiles.size() * sizeof(TrsmTile)));
  HIP_TRY(launch_trsm_f64((const TrsmItem *)h->ws_items.p, (const TrsmTile *)h->ws_tiles.p, nct, 0));
  // BF16 hi/lo copies in fragment layouts
  h->wa_off_h.resize(h->nblk);
  h->wb_off_h.resize(h->nblk);
  int64_t wa = 0, wb = 0, max_k = 0;
  for (int32_t i = 0; i < h->nblk; ++i) {
    const int64_t ka = (int64_t)(i + 1 - h->blk_first_h[i]) * TB;
    const int64_t kb = (int64_t)(h->blk_last_h[i] + 1 - i) * TB;
    h->wa_off_h[i] = wa;
    h->wb_off_h[i] = wb;
    wa += ka * TB;
    wb += kb * TB;
    max_k = std::max(max_k, std::max(ka, kb));
  }
  TDA_TRY(upload(h, h->wa_off_d, h->wa_off_h.data(), h->nblk * sizeof(int64_t)));
  TDA_TRY(upload(h, h->wb_off_d, h->wb_off_h.data(), h->nblk * sizeof(int64_t)));
  TDA_TRY(h->alloc(h->wa_hi, (size_t)wa * 2));
  TDA_TRY(h->alloc(h->wa_lo, (size_t)wa * 2));
  TDA_TRY(h->alloc(h->wb_hi, (size_t)wb * 2));
  TDA_TRY(h->alloc(h->wb_lo, (size_t)wb * 2));
  HIP_TRY(launch_split_w((const double *)h->w64_d.p, (const int64_t *)h->w64_off_d.p,
                         (const int32_t *)h->w64_rb_d.p, (const int32_t *)h->blk_first_d.p,
                         (const int32_t *)h->blk_last_d.p, h->nblk, (uint16_t *)h->wa_hi.p,
                         (uint16_t *)h->wa_lo.p, (const int64_t *)h->wa_off_d.p,
                         (uint16_t *)h->wb_hi.p, (uint16_t *)h->wb_lo.p,
                         (const int64_t *)h->wb_off_d.p, max_k, 0, 0));
  // circulant eigenvalues and twiddles per segment
  // (per segment: m eigenvalues; m twiddles w_m^r then m/4 pass twiddles, complex)
  int64_t msum = 0;
  for (const Seg &g : h->segs) msum += g.m;
  TDA_TRY(h->alloc(h->lam_d, (size_t)msum * sizeof(double)));
  TDA_TRY(h->alloc(h->tw_d, (size_t)2 * (msum + msum / 4) * sizeof(double)));
  h->segdev_h.clear();
  int64_t mo = 0;
  for (const Seg &g : h->segs) {
    double *lam = (double *)h->lam_d.p + mo;
    double *tw = (double *)h->tw_d.p + 2 * (mo + mo / 4);
    double *ptw = tw + 2 * g.m;
    HIP_TRY(launch_lambda((const double *)h->acf_d.p, g.length, g.m, tw, lam, ptw, 0));
    SegDev sd{};
    sd.offset = g.offset;
    sd.length = g.length;
    sd.row0 = g.row0;
    sd.nkeep = g.n_keep;
    sd.npad = g.n_pad;
    sd.m = g.m;
    sd.log2m = g.log2m;
    sd.lam = lam;
    sd.tw = tw;
    sd.ptw = ptw;
    h->segdev_h.push_back(sd);
    h->max_m = std::max(h->max_m, g.m);
    mo += g.m;
  }
  TDA_TRY(upload(h, h->segdev_d, h->segdev_h.data(), h->segdev_h.size() * sizeof(SegDev)));
  // whitened-data cache (invalid until the first data check) and the per-call check
  TDA_TRY(h->alloc(h->cache_d, sizeof(DataCache)));
  TDA_TRY(h->alloc(h->chk_d, sizeof(DataCheck)));
  HIP_TRY(hipMemset(h->cache_d.p, 0, sizeof(DataCache)));
  HIP_TRY(hipMemset(h->chk_d.p, 0, sizeof(DataCheck)));
  HIP_TRY(hipDeviceSynchronize());
  return TDA_OK;
}

// Enqueue the data check of a mixed handle for data d into chk (device): the fingerprint
// of d's retained samples against the cached one and, while the handle holds its FP64
// operator, the whitening kernels, which run only on a mismatch (or with force).  A
// compact handle cannot whiten new data: the check then sets chk->qdd to NaN.
static tda_status enqueue_data_check(tda_ctx *h, const double *d, DataCheck *chk, bool force,
                                     hipStream_t s) {
  const bool can_whiten = !h->compacted && h->w64_d.p;
  if (can_whiten) {
    TDA_TRY(h->alloc(h->dbar_d, (size_t)h->n_pad * sizeof(double)));
    TDA_TRY(h->alloc(h->yd_d, (size_t)h->n_pad * sizeof(double)));
    TDA_TRY(h->alloc(h->ydpos_d, (size_t)h->N * sizeof(double)));
  }
  {
    TimedScope ts("data_check", s);
    HIP_TRY(launch_data_check(d, (const int32_t *)h->idx_d.p, (int32_t)h->n_pad,
                              (DataCache *)h->cache_d.p, chk, can_whiten ? 1 : 0, force ? 1 : 0, s));
  }
  if (can_whiten) {
    TimedScope ts("data_whiten", s);
    HIP_TRY(launch_data_whiten((const double *)h->w64_d.p, (const int64_t *)h->w64_off_d.p,
                               (const int32_t *)h->w64_rb_d.p, (const int32_t *)h->blk_first_d.p,
                               (const int32_t *)h->blk_last_d.p, (const int32_t *)h->idx_d.p,
                               (const int32_t *)h->pos2row_d.p, (int32_t)h->n_pad, h->N, d,
                               (double *)h->dbar_d.p, (double *)h->yd_d.p,
                               (double *)h->ydpos_d.p, (DataCache *)h->cache_d.p, chk, s));
  }
  return TDA_OK;
}

// Whiten d now (tda_set_data, server registration); a compact handle then releases its
// FP64 operator and solve panels.
static tda_status set_data_impl(tda_ctx *h, const double *d, hipStream_t s) {
  if (h->compacted)
    return fail_with(TDA_ESTATE, "compact handle: the FP64 operator was released after its data");
  TDA_TRY(enqueue_data_check(h, d, (DataCheck *)h->chk_d.p, true, s));
  h->data_ptr = d;
  if (h->flags & TDA_FLAG_COMPACT) {
    HIP_TRY(hipStreamSynchronize(s));
    h->release(h->w64_d);
    h->release(h->panels_d);
    h->release(h->dbar_d);
    h->release(h->yd_d);
    h->compacted = true;
  }
  return TDA_OK;
}

extern "C" tda_status tda_set_data(tda_handle h, const double *d, void *hip_stream) {
  if (!h) return fail_with(TDA_EINVAL, "NULL handle");
  if (!h->factored) return fail_with(TDA_ESTATE, "tda_set_data before tda_factor");
  if (!d) return fail_with(TDA_EINVAL, "NULL data");
  if (h->precision != TDA_PREC_MIXED) return TDA_OK;
  DeviceGuard guard(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  TDA_TRY(order_after_previous(h, s));
  TDA_TRY(set_data_impl(h, d, s));
  return mark_done(h, s);
}

// Per-call operand workspace of one mixed item.
struct MixWs {
  uint16_t *hs_hi, *hs_lo, *w0_hi, *w0_lo;
  float *y0;
  double *e64, *qpart, *corr_part;
};

// Bytes of workspace one mixed item needs for Bp templates.
// fragments per template tile of the split layouts
static int64_t tile_ksteps(const tda_ctx *h) { return h->n_pad / 16 + TKS_PAD; }

// Segments whose circulant the refinement splits into halves or quarters park part of
// C y0 in an FP64 scratch row per template.
static bool needs_e64(const tda_ctx *h) {
  return h->max_m > RL_MAX_M && h->max_m <= RL_MAX_M_QUAD;
}

static size_t mix_ws_bytes(const tda_ctx *h, int64_t Bp) {
  const size_t el = (size_t)Bp * h->n_pad;
  const size_t el_t = (size_t)(Bp / 32) * tile_ksteps(h) * 512;  // split layouts
  return el_t * (2 + 2 + 2 + 2) + el * (4 + (needs_e64(h) ? 8 : 0)) + (size_t)Bp * 8 +
         (size_t)h->nblk * Bp * 8 + 6 * 256;
}

static MixWs carve_mix_ws(const tda_ctx *h, int64_t Bp, char *base) {
  const size_t el = (size_t)Bp * h->n_pad;
  const size_t el_t = (size_t)(Bp / 32) * tile_ksteps(h) * 512;
  auto take = [&](size_t bytes) {
    char *p = base;
    base += (bytes + 255) & ~(size_t)255;
    return p;
  };
  MixWs w;
  w.hs_hi = (uint16_t *)take(el_t * 2);
  w.hs_lo = (uint16_t *)take(el_t * 2);
  w.w0_hi = (uint16_t *)take(el_t * 2);
  w.w0_lo = (uint16_t *)take(el_t * 2);
  w.y0 = (float *)take(el * 4);
  w.e64 = needs_e64(h) ? (double *)take(el * 8) : nullptr;
  w.qpart = (double *)take((size_t)Bp * 8);
  w.corr_part = (double *)take((size_t)h->nblk * Bp * 8);
  return w;
}

static MixItem make_mix_item(const tda_ctx *h, const double *H, int64_t ldh, int64_t B,
                             int64_t Bp, const MixWs &ws, double *out) {
  MixItem mi{};
  mi.wa_hi = (const uint16_t *)h->wa_hi.p;
  mi.wa_lo = (const uint16_t *)h->wa_lo.p;
  mi.wb_hi = (const uint16_t *)h->wb_hi.p;
  mi.wb_lo = (const uint16_t *)h->wb_lo.p;
  mi.wa_off = (const int64_t *)h->wa_off_d.p;
  mi.wb_off = (const int64_t *)h->wb_off_d.p;
  mi.blk_first = (const int32_t *)h->blk_first_d.p;
  mi.blk_last = (const int32_t *)h->blk_last_d.p;
  mi.idx = (const int32_t *)h->idx_d.p;
  mi.H = H;
  mi.ldh = ldh;
  mi.hs_hi = ws.hs_hi;
  mi.hs_lo = ws.hs_lo;
  mi.es_hi = ws.hs_hi;  // the residual's split reuses the buffer once the products are done
  mi.es_lo = ws.hs_lo;
  mi.w0_hi = ws.w0_hi;
  mi.w0_lo = ws.w0_lo;
  mi.y0 = ws.y0;
  mi.e64 = ws.e64;
  mi.corr_part = ws.corr_part;
  mi.qpart = ws.qpart;
  mi.out = out;
  mi.cterm = h->cterm();
  mi.B = (int32_t)B;
  mi.Bp = (int32_t)Bp;
  mi.nblk = h->nblk;
  mi.n_pad = (int32_t)h->n_pad;
  mi.tks = tile_ksteps(h);
  return mi;
}

static RefItem make_ref_item(const tda_ctx *h, const MixItem &mi, const DataCheck *chk) {
  RefItem ri{};
  ri.segs = (const SegDev *)h->segdev_d.p;
  ri.n_segs = (int32_t)h->segdev_h.size();
  ri.B = mi.B;
  ri.pos2row = (const int32_t *)h->pos2row_d.p;
  ri.y0 = mi.y0;
  ri.H = mi.H;
  ri.ldh = mi.ldh;
  ri.Hrows = mi.Hrows;
  ri.yd_pos = (const double *)h->ydpos_d.p;
  ri.qdd = &chk->qdd;
  ri.idx = (const int32_t *)h->idx_d.p;
  ri.e64 = mi.e64;
  ri.es_hi = mi.es_hi;
  ri.es_lo = mi.es_lo;
  ri.tks = mi.tks;
  ri.qpart = mi.qpart;
  ri.out = mi.out;
  ri.cterm = mi.cterm;
  ri.n_pad = mi.n_pad;
  return ri;
}

// Refinement work: templates of one item in pairs sharing one complex DFT.
static void add_refine_pairs(int32_t item, int64_t B, std::vector<int4> &wr) {
  for (int64_t b = 0; b < B; b += 2)
    wr.push_back(int4{item, (int32_t)b, b + 1 < B ? (int32_t)(b + 1) : -1, 0});
}

// product jobs: (block pair, template group, half); see the product kernels for pairs
// and halves.  A job is named by the first block of its pair, the lower index; its
// weight is the K the pair spans, the same for both products.
static void add_block_jobs(const tda_ctx *h, int32_t item, int32_t ntg, int32_t nsub,
                           std::vector<BlockJob> &jobs) {
  for (int32_t i = 0; i < h->nblk; ++i) {
    const int32_t bf = h->blk_first_h[i], bl = h->blk_last_h[i], partner = bf + bl - i;
    if (partner < i) continue;  // second block of a pair
    const int64_t k = partner == i ? (int64_t)(i + 1 - bf) : (int64_t)(bl - bf + 2);
    jobs.push_back(BlockJob{item, i, ntg, nsub, k});
  }
}

// Product variants whose workgroup covers a whole group of 256 templates take the work
// list without halves: an entry that exits at once still holds a dispatch slot of its
// CU, and half of such entries left half of the CUs idle.
static bool variant_full_group(int v) { return v != 2; }

// timing names carry the product variant the autotuner picked ("trmm_fwd/v2")
static const char *const kTrmmFwdNames[] = {"trmm_fwd",    "trmm_fwd/v1", "trmm_fwd/v2",
                                            "trmm_fwd/v3", "trmm_fwd/v4", "trmm_fwd/v5"};
static const char *const kTrmmBwdNames[] = {"trmm_bwd",    "trmm_bwd/v1", "trmm_bwd/v2",
                                            "trmm_bwd/v3", "trmm_bwd/v4", "trmm_bwd/v5"};
static const char *const kTrmmCorrNames[] = {"trmm_corr",    "trmm_corr/v1", "trmm_corr/v2",
                                             "trmm_corr/v3", "trmm_corr/v4", "trmm_corr/v5"};
static const char *variant_name(const char *const *names, int v) {
  return v >= 1 && v <= 5 ? names[v] : names[0];
}

// The mixed launch sequence over a set of items whose MixItem/RefItem descriptors are
// already built (host side); descriptors and work lists go through `ring` on stream s.
static tda_status enqueue_mixed(DescRing &ring, const std::vector<MixItem> &mis,
                                const std::vector<RefItem> &ris,
                                const std::vector<const tda_ctx *> &hs, double *fft_scratch,
                                int64_t max_m, hipStream_t s) {
  const int64_t n = (int64_t)mis.size();
  // refinement in LDS for items whose segments' circulants fit, paired with global
  // scratch for the others
  (void)max_m;
  std::vector<BlockJob> jf, jh;
  std::vector<int4> wr;
  std::vector<int2> wfin, wrl;
  for (int64_t k = 0; k < n; ++k) {
    if (mis[k].B == 0) continue;
    add_block_jobs(hs[k], (int32_t)k, mis[k].Bp / 256, 1, jf);
    add_block_jobs(hs[k], (int32_t)k, mis[k].Bp / 256, 2, jh);
    const bool in_lds = hs[k]->max_m <= RL_MAX_M_QUAD;
    if (!in_lds) add_refine_pairs((int32_t)k, mis[k].B, wr);
    for (int32_t b = 0; b < mis[k].B; ++b) {
      wfin.push_back(int2{(int32_t)k, b});
      if (in_lds) wrl.push_back(int2{(int32_t)k, b});
    }
  }
  int64_t max_m_scratch = 0;
  for (int64_t k = 0; k < n; ++k)
    if (mis[k].B > 0 && hs[k]->max_m > RL_MAX_M_QUAD) max_m_scratch = std::max(max_m_scratch, hs[k]->max_m);
  // quarter-split segments keep three quarters of their transforms in the same scratch
  bool quad = false;
  for (int64_t k = 0; k < n; ++k)
    quad |= mis[k].B > 0 && hs[k]->max_m > RL_MAX_M_SPLIT && hs[k]->max_m <= RL_MAX_M_QUAD;
  // the forward, backward and correction products share the work lists (block pairs):
  // whole template groups, and half groups for the half-group variant
  const std::vector<int4> wf = xcd_order(jf), wh = xcd_order(jh);
  wrl = xcd_tiles(wrl);
  HIP_TRY(ring.reserve(8192 + n * (64 + sizeof(MixItem) + sizeof(RefItem)) +
                       (wf.size() + wh.size() + wr.size()) * sizeof(int4) +
                       (wfin.size() + wrl.size()) * sizeof(int2)));
  void *d_mi, *d_ri, *d_wf, *d_wh, *d_wr, *d_fin, *d_rl = nullptr;
  HIP_TRY(ring.push(mis.data(), mis.size() * sizeof(MixItem), s, &d_mi));
  HIP_TRY(ring.push(ris.data(), ris.size() * sizeof(RefItem), s, &d_ri));
  HIP_TRY(ring.push(wf.data(), wf.size() * sizeof(int4), s, &d_wf));
  HIP_TRY(ring.push(wh.data(), wh.size() * sizeof(int4), s, &d_wh));
  d_wr = nullptr;
  if (!wr.empty()) HIP_TRY(ring.push(wr.data(), wr.size() * sizeof(int4), s, &d_wr));
  HIP_TRY(ring.push(wfin.data(), wfin.size() * sizeof(int2), s, &d_fin));
  if (!wrl.empty()) HIP_TRY(ring.push(wrl.data(), wrl.size() * sizeof(int2), s, &d_rl));
  const MixItem *dm = (const MixItem *)d_mi;
  // autotuned variant per product kernel, keyed by the largest item's shape
  int64_t rows = 0, tmpl = 0;
  for (int64_t k = 0; k < n; ++k) {
    rows = std::max<int64_t>(rows, mis[k].n_pad);
    tmpl += mis[k].Bp;
  }
  struct Ctx {
    const MixItem *dm;
    const int4 *wf, *wh;  // whole-group and half-group work lists
    int64_t nf, nh;
    hipStream_t s;
    const int4 *w(int v) const { return variant_full_group(v) ? wf : wh; }
    int64_t nw(int v) const { return variant_full_group(v) ? nf : nh; }
  };
  static const int kVariants[4] = {1, 2, 4, 5};
  Ctx cf{dm, (const int4 *)d_wf, (const int4 *)d_wh, (int64_t)wf.size(), (int64_t)wh.size(), s};
  int64_t max_chunks = 0;
  for (int64_t k = 0; k < n; ++k)
    max_chunks = std::max<int64_t>(max_chunks, (int64_t)(mis[k].Bp / 32) * (mis[k].n_pad / 16) * 64);
  {
    TimedScope ts("split_h", s);
    HIP_TRY(launch_split_h(dm, (int32_t)n, max_chunks, s));
  }
  const int vf = autotune_pick("trmm_fwd", rows, tmpl, kVariants, 4, s,
                               [](void *c, int v) {
                                 Ctx *x = (Ctx *)c;
                                 return launch_trmm_fwd(x->dm, x->w(v), x->nw(v), v, x->s);
                               }, &cf);
  {
    TimedScope ts(variant_name(kTrmmFwdNames, vf), s);
    HIP_TRY(launch_trmm_fwd(dm, cf.w(vf), cf.nw(vf), vf, s));
  }
  const int vb = autotune_pick("trmm_bwd", rows, tmpl, kVariants, 4, s,
                               [](void *c, int v) {
                                 Ctx *x = (Ctx *)c;
                                 return launch_trmm_bwd(x->dm, x->w(v), x->nw(v), v, x->s);
                               }, &cf);
  {
    TimedScope ts(variant_name(kTrmmBwdNames, vb), s);
    HIP_TRY(launch_trmm_bwd(dm, cf.w(vb), cf.nw(vb), vb, s));
  }
  {
    TimedScope ts("refine_fft", s);
    if (!wrl.empty())
      HIP_TRY(launch_refine_lds((const RefItem *)d_ri, (const int2 *)d_rl, (int64_t)wrl.size(),
                                quad ? fft_scratch : nullptr, s));
    if (!wr.empty())
      HIP_TRY(launch_refine((const RefItem *)d_ri, (const int4 *)d_wr, (int64_t)wr.size(),
                            fft_scratch, 2 * max_m_scratch, kRefineWG, s));
  }
  const int vc = autotune_pick("trmm_corr", rows, tmpl, kVariants, 4, s,
                               [](void *c, int v) {
                                 Ctx *x = (Ctx *)c;
                                 return launch_corr(x->dm, x->w(v), x->nw(v), v, x->s);
                               }, &cf);
  {
    TimedScope ts(variant_name(kTrmmCorrNames, vc), s);
    HIP_TRY(launch_corr(dm, cf.w(vc), cf.nw(vc), vc, s));
  }
  {
    TimedScope ts("finish", s);
    HIP_TRY(launch_finish(dm, (const int2 *)d_fin, (int64_t)wfin.size(), s));
  }
  return TDA_OK;
}

// Explicit-inverse FP64 evaluation: residual rows packed per template, one FP64
// matrix-core product per (block pair, 64 templates) against the FP64 W = L^-1 of the
// mixed handle, block sums of squares added in block order.
static tda_status loglik_cdo(tda_ctx *h, const double *d, const double *H, int64_t B,
                             int64_t ldh, double *out, hipStream_t s) {
  const int64_t Bp = (B + CDO_T - 1) / CDO_T * CDO_T;
  const size_t r_bytes = (size_t)Bp * h->n_pad * sizeof(double);
  TDA_TRY(h->alloc(h->ws_cdo, r_bytes + (size_t)h->nblk * Bp * sizeof(double)));
  CdoItem it{};
  it.w64 = (const double *)h->w64_d.p;
  it.w64_off = (const int64_t *)h->w64_off_d.p;
  it.w64_rb = (const int32_t *)h->w64_rb_d.p;
  it.blk_first = (const int32_t *)h->blk_first_d.p;
  it.blk_last = (const int32_t *)h->blk_last_d.p;
  it.idx = (const int32_t *)h->idx_d.p;
  it.d = d;
  it.H = H;
  it.ldh = ldh;
  it.R = (double *)h->ws_cdo.p;
  it.part = (double *)((char *)h->ws_cdo.p + r_bytes);
  it.out = out;
  it.cterm = h->cterm();
  it.B = (int32_t)B;
  it.Bp = (int32_t)Bp;
  it.nblk = h->nblk;
  it.n_pad = (int32_t)h->n_pad;
  std::vector<BlockJob> jobs;
  add_block_jobs(h, 0, (int32_t)(Bp / CDO_T), 1, jobs);
  const std::vector<int4> work = xcd_order(jobs);
  HIP_TRY(h->ring.reserve(1024 + sizeof(CdoItem) + work.size() * sizeof(int4)));
  void *d_it, *d_w;
  HIP_TRY(h->ring.push(&it, sizeof(CdoItem), s, &d_it));
  HIP_TRY(h->ring.push(work.data(), work.size() * sizeof(int4), s, &d_w));
  {
    TimedScope ts("cdo_pack", s);
    HIP_TRY(launch_cdo_pack((const CdoItem *)d_it, it, s));
  }
  {
    TimedScope ts("cdo_f64", s);
    HIP_TRY(launch_cdo((const CdoItem *)d_it, (const int4 *)d_w, (int64_t)work.size(), s));
  }
  HIP_TRY(launch_cdo_finish((const CdoItem *)d_it, B, s));
  HIP_TRY(h->ring.seal(s));
  return TDA_OK;
}

static tda_status loglik_mixed(tda_ctx *h, const double *d, const double *H, int64_t B,
                               int64_t ldh, double *out, hipStream_t s, double *out_dh,
                               double *out_hh) {
  DataCheck *chk = (DataCheck *)h->chk_d.p;
  TDA_TRY(enqueue_data_check(h, d, chk, false, s));
  h->data_ptr = d;
  const int64_t Bp = (B + MT - 1) / MT * MT;
  TDA_TRY(h->alloc(h->ws_mix, mix_ws_bytes(h, Bp)));
  if (fft_ws_bytes(h->max_m)) TDA_TRY(h->alloc(h->ws_fft, fft_ws_bytes(h->max_m)));
  const MixWs ws = carve_mix_ws(h, Bp, (char *)h->ws_mix.p);
  std::vector<MixItem> mis{make_mix_item(h, H, ldh, B, Bp, ws, out)};
  mis[0].hh_out = out_hh;
  std::vector<RefItem> ris{make_ref_item(h, mis[0], chk)};
  ris[0].dh_out = out_dh;
  ris[0].hh_out = out_hh;
  std::vector<const tda_ctx *> hs{h};
  TDA_TRY(enqueue_mixed(h->ring, mis, ris, hs, (double *)h->ws_fft.p, h->max_m, s));
  HIP_TRY(h->ring.seal(s));
  return TDA_OK;
}

// ---------------------------------------------------------------- batched multi-item evaluation

namespace {

}  // namespace

struct tda::MultiCtx {
  std::mutex mu;
  tda_ctx pool;  // used only for its allocator and buffers
  DescRing ring;
  hipEvent_t done = nullptr;
};

namespace {

MultiCtx *multi_ctx(int dev) {
  static std::mutex g;
  static std::vector<MultiCtx *> ctxs;
  std::lock_guard<std::mutex> lk(g);
  if ((int)ctxs.size() <= dev) ctxs.resize(dev + 1, nullptr);
  if (!ctxs[dev]) ctxs[dev] = new MultiCtx();
  return ctxs[dev];
}

tda_status multi_impl(MultiCtx *mc, const tda_work *items, const double *const *const *hrows,
                      int64_t n_items, int32_t precision, hipStream_t s, bool order_handles);

}  // namespace

namespace tda {
MultiCtx *multi_ctx_create() { return new MultiCtx(); }
void multi_ctx_destroy(MultiCtx *mc) {
  if (!mc) return;
  mc->pool.release_all();
  mc->ring.destroy();
  if (mc->done) (void)hipEventDestroy(mc->done);
  delete mc;
}
tda_status multi_eval(MultiCtx *mc, const tda_work *items, const double *const *const *hrows,
                      int64_t n_items, int32_t precision, hipStream_t s) {
  return multi_impl(mc, items, hrows, n_items, precision, s, false);
}
size_t item_ws_bytes(tda_handle h, int64_t B, int32_t precision) {
  if (B <= 0) return 0;
  if (precision == TDA_PREC_MIXED) return mix_ws_bytes(h, (B + MT - 1) / MT * MT);
  if (precision == TDA_PREC_FP64)
    return (size_t)((B + BC - 1) / BC) * (size_t)h->n_pad * BC * sizeof(double);
  return 0;
}
size_t launch_ws_fixed_bytes(tda_handle h, int32_t precision) {
  return precision == TDA_PREC_MIXED ? fft_ws_bytes(h->max_m) : 0;
}
size_t multi_ctx_held(MultiCtx *mc) { return mc ? mc->pool.held : 0; }
int handle_device(tda_handle h) { return h->device; }
int64_t handle_n(tda_handle h) { return h->N; }
size_t handle_bytes(tda_handle h) { return h->held; }
bool handle_ready(tda_handle h, int32_t precision) {
  if (!h->factored) return false;
  if ((precision == TDA_PREC_GS) != (h->precision == TDA_PREC_GS)) return false;
  if (precision == TDA_PREC_FP64) return !h->compacted;
  return h->precision == precision;
}
tda_status handle_set_data(tda_handle h, const double *d, hipStream_t s) {
  if (h->precision != TDA_PREC_MIXED) return TDA_OK;
  if (h->compacted)
    return h->data_ptr == d ? TDA_OK
                            : fail_with(TDA_ESTATE, "compact handle: data other than its cached data");
  return set_data_impl(h, d, s);
}
const double *handle_data(tda_handle h) { return h->data_ptr; }
tda_status set_error(tda_status st, const char *msg) { return fail_with(st, "%s", msg); }
}  // namespace tda

extern "C" tda_status tda_loglik_multi(const tda_work *items, int64_t n_items, int32_t precision,
                                       void *hip_stream) {
  if (n_items < 0 || (n_items > 0 && !items)) return fail_with(TDA_EINVAL, "bad item list");
  if (n_items == 0) return TDA_OK;
  if (!items[0].h) return fail_with(TDA_EINVAL, "item 0: NULL handle");
  MultiCtx *mc = multi_ctx(items[0].h->device);
  std::lock_guard<std::mutex> lk(mc->mu);
  DeviceGuard guard(items[0].h->device);
  return multi_impl(mc, items, nullptr, n_items, precision, (hipStream_t)hip_stream, true);
}

extern "C" tda_status tda_release_workspaces(int32_t device) {
  int dev = device, n_dev = 0;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail_with(TDA_EHIP, "hipGetDevice failed");
  if (hipGetDeviceCount(&n_dev) != hipSuccess || dev >= n_dev)
    return fail_with(TDA_EINVAL, "device %d out of range", dev);
  MultiCtx *mc = multi_ctx(dev);
  std::lock_guard<std::mutex> lk(mc->mu);
  DeviceGuard guard(dev);
  // earlier batched calls may still be running on their streams
  HIP_TRY(hipDeviceSynchronize());
  mc->pool.release_all();
  return TDA_OK;
}

namespace {
tda_status multi_impl(MultiCtx *mc, const tda_work *items, const double *const *const *hrows,
                      int64_t n_items, int32_t precision, hipStream_t s, bool order_handles) {
  if (n_items == 0) return TDA_OK;
  if (precision == TDA_PREC_CDO)
    return fail_with(TDA_EINVAL, "explicit-inverse evaluation is per handle (tda_loglik_ex)");
  if (precision != TDA_PREC_FP64 && precision != TDA_PREC_MIXED && precision != TDA_PREC_GS)
    return fail_with(TDA_EINVAL, "unknown precision");
  const int dev = items[0].h ? items[0].h->device : -1;
  std::vector<double *> group_out;
  std::vector<int64_t> group_B;
  std::vector<int32_t> group_of(n_items);
  std::vector<int64_t> part_off(n_items);
  int64_t parts = 0, max_B = 0;
  for (int64_t k = 0; k < n_items; ++k) {
    const tda_work &w = items[k];
    if (!w.h) return fail_with(TDA_EINVAL, "item %lld: NULL handle", (long long)k);
    if (!w.h->factored) return fail_with(TDA_ESTATE, "item %lld: handle not factored", (long long)k);
    if (w.h->device != dev) return fail_with(TDA_EINVAL, "items on different devices");
    if (w.B < 0 || w.B > ((int64_t)1 << 30)) return fail_with(TDA_EINVAL, "item %lld: bad B", (long long)k);
    if (w.B > 0 && (!w.d || !(w.H || (hrows && hrows[k])) || !w.out))
      return fail_with(TDA_EINVAL, "item %lld: NULL pointer", (long long)k);
    if (w.ldh < w.h->N) return fail_with(TDA_EINVAL, "item %lld: ldh < N", (long long)k);
    if (precision == TDA_PREC_MIXED && w.h->precision != TDA_PREC_MIXED)
      return fail_with(TDA_ESTATE, "item %lld: handle not built for mixed precision", (long long)k);
    if ((precision == TDA_PREC_GS) != (w.h->precision == TDA_PREC_GS))
      return fail_with(TDA_ESTATE, "item %lld: GS handles evaluate only (and only they) in GS",
                       (long long)k);
    if (w.h->compacted && (precision == TDA_PREC_FP64 || w.d != w.h->data_ptr))
      return fail_with(TDA_ESTATE, "item %lld: compact handle used beyond its cached data",
                       (long long)k);
    int32_t g = -1;
    for (size_t q = 0; q < group_out.size(); ++q)
      if (group_out[q] == w.out) g = (int32_t)q;
    if (g < 0) {
      g = (int32_t)group_out.size();
      group_out.push_back(w.out);
      group_B.push_back(w.B);
    } else if (group_B[g] != w.B) {
      return fail_with(TDA_EINVAL, "items sharing an output must have equal B");
    }
    group_of[k] = g;
    part_off[k] = parts;
    parts += w.B;
    max_B = std::max(max_B, w.B);
    if (precision == TDA_PREC_MIXED)
      for (int64_t q = 0; q < k; ++q)
        if (items[q].h == w.h && items[q].d != w.d)
          return fail_with(TDA_EINVAL, "one handle used with two data vectors in one call");
  }
  if (max_B == 0) return TDA_OK;
  tda_ctx &P = mc->pool;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cap));
  const bool capturing = cap == hipStreamCaptureStatusActive;
  if (capturing && !mc->ring.graph)
    return fail_with(TDA_ESTATE, "stream capture outside a plan: use tda_plan_execute");
  if (!mc->done) HIP_TRY(hipEventCreateWithFlags(&mc->done, hipEventDisableTiming));
  if (!capturing) HIP_TRY(hipStreamWaitEvent(s, mc->done, 0));
  for (int64_t k = 0; k < n_items; ++k)
    if (order_handles) TDA_TRY(order_after_previous(items[k].h, s));
  // partial results, then one data check per item (items of one handle share the first's)
  const size_t part_bytes = ((size_t)parts * sizeof(double) + 255) & ~(size_t)255;
  TDA_TRY(P.alloc(P.ws_work, part_bytes + (size_t)n_items * sizeof(DataCheck)));
  double *partbuf = (double *)P.ws_work.p;
  DataCheck *chks = (DataCheck *)((char *)P.ws_work.p + part_bytes);
  std::vector<int64_t> chk_of(n_items, -1);
  if (precision == TDA_PREC_MIXED)
    for (int64_t k = 0; k < n_items; ++k) {
      if (items[k].B == 0) continue;
      for (int64_t q = 0; q < k && chk_of[k] < 0; ++q)
        if (items[q].h == items[k].h && chk_of[q] >= 0) chk_of[k] = chk_of[q];
      if (chk_of[k] >= 0) continue;
      chk_of[k] = k;
      TDA_TRY(enqueue_data_check(items[k].h, items[k].d, chks + k, false, s));
      items[k].h->data_ptr = items[k].d;
    }
  std::vector<void *> blobs;
  if (precision == TDA_PREC_GS) {
    std::vector<GsItem> gis(n_items);
    std::vector<int2> work;
    int64_t max_len = 0, max_m = 0;
    for (int64_t k = 0; k < n_items; ++k) {
      const tda_work &w = items[k];
      gis[k] = make_gs_item(w.h, w.d, w.H, w.ldh, w.B, partbuf + part_off[k]);
      gis[k].Hrows = hrows ? hrows[k] : nullptr;
      max_len = std::max(max_len, w.h->gs_max_len);
      max_m = std::max(max_m, w.h->max_m);
      for (int64_t b = 0; b < w.B; ++b) work.push_back(int2{(int32_t)k, (int32_t)b});
    }
    work = xcd_tiles(work);
    const GsScratch gsc = gs_scratch_plan((int64_t)work.size(), max_len, max_m);
    TDA_TRY(P.alloc(P.ws_fft, gsc.bytes));
    HIP_TRY(mc->ring.reserve(4096 + gis.size() * sizeof(GsItem) + work.size() * sizeof(int2) +
                             n_items * 16 + group_out.size() * 16));
    void *d_it, *d_w;
    HIP_TRY(mc->ring.push(gis.data(), gis.size() * sizeof(GsItem), s, &d_it));
    HIP_TRY(mc->ring.push(work.data(), work.size() * sizeof(int2), s, &d_w));
    TimedScope ts("gs_fft", s);
    HIP_TRY(launch_gs((const GsItem *)d_it, (const int2 *)d_w, (int64_t)work.size(),
                      (double *)P.ws_fft.p, gsc.stride, gsc.qoff, gsc.n_wg, s));
  } else if (precision == TDA_PREC_FP64) {
    std::vector<TrsmItem> its(n_items);
    std::vector<TrsmTile> tiles;
    int64_t scratch = 0;
    for (int64_t k = 0; k < n_items; ++k) {
      const tda_work &w = items[k];
      tda_ctx *h = w.h;
      TrsmItem &it = its[k];
      it.panels = (const double *)h->panels_d.p;
      it.panel_off = (const int64_t *)h->panel_off_d.p;
      it.blk_first = (const int32_t *)h->blk_first_d.p;
      it.idx = (const int32_t *)h->idx_d.p;
      it.d = w.d;
      it.H = w.H;
      it.ldh = w.ldh;
      it.Hrows = hrows ? hrows[k] : nullptr;
      it.out = partbuf + part_off[k];
      it.cterm = h->cterm();
      it.B = (int32_t)w.B;
      it.mode = MODE_LOGLIK;
      const int64_t nt = (w.B + BC - 1) / BC;
      for (int64_t t = 0; t < nt; ++t)
        tiles.push_back(TrsmTile{(int32_t)k, (int32_t)(t * BC), 0, h->nblk,
                                 scratch + t * h->n_pad * BC});
      it.scratch = (double *)(intptr_t)scratch;  // offset; rebased below
      scratch += nt * h->n_pad * BC;
    }
    TDA_TRY(P.alloc(P.ws_scratch, (size_t)scratch * sizeof(double)));
    for (int64_t k = 0; k < n_items; ++k) its[k].scratch = (double *)P.ws_scratch.p;
    // longest sweeps first
    std::stable_sort(tiles.begin(), tiles.end(), [&](const TrsmTile &a, const TrsmTile &b) {
      return items[a.item].h->n_pad > items[b.item].h->n_pad;
    });
    HIP_TRY(mc->ring.reserve(2048 + its.size() * sizeof(TrsmItem) + tiles.size() * sizeof(TrsmTile) +
                             n_items * 16 + group_out.size() * 16));
    void *d_its, *d_tiles;
    HIP_TRY(mc->ring.push(its.data(), its.size() * sizeof(TrsmItem), s, &d_its));
    HIP_TRY(mc->ring.push(tiles.data(), tiles.size() * sizeof(TrsmTile), s, &d_tiles));
    TimedScope ts("trsm_f64", s);
    HIP_TRY(launch_trsm_f64((const TrsmItem *)d_its, (const TrsmTile *)d_tiles,
                            (int64_t)tiles.size(), s));
  } else {
    std::vector<MixItem> mis(n_items);
    std::vector<RefItem> ris(n_items);
    std::vector<const tda_ctx *> hs(n_items);
    size_t total = 0;
    int64_t max_m = 0;
    std::vector<size_t> ws_off(n_items);
    for (int64_t k = 0; k < n_items; ++k) {
      const int64_t Bp = (items[k].B + MT - 1) / MT * MT;
      ws_off[k] = total;
      total += mix_ws_bytes(items[k].h, Bp);
      max_m = std::max(max_m, items[k].h->max_m);
    }
    TDA_TRY(P.alloc(P.ws_mix, total));
    if (fft_ws_bytes(max_m)) TDA_TRY(P.alloc(P.ws_fft, fft_ws_bytes(max_m)));
    for (int64_t k = 0; k < n_items; ++k) {
      const tda_work &w = items[k];
      const int64_t Bp = (w.B + MT - 1) / MT * MT;
      const MixWs ws = carve_mix_ws(w.h, Bp, (char *)P.ws_mix.p + ws_off[k]);
      mis[k] = make_mix_item(w.h, w.H, w.ldh, w.B, Bp, ws, partbuf + part_off[k]);
      mis[k].Hrows = hrows ? hrows[k] : nullptr;
      ris[k] = make_ref_item(w.h, mis[k], chks + std::max<int64_t>(chk_of[k], 0));
      hs[k] = w.h;
    }
    // detectors that evaluate the same templates over the same padded rows share one
    // template split: the split pass runs once and the forward products read one copy
    for (int64_t k = 1; k < n_items; ++k)
      for (int64_t j = 0; j < k; ++j) {
        const MixItem &a = mis[j];
        MixItem &b = mis[k];
        if (a.hs_shared || a.H != b.H || a.ldh != b.ldh || a.Hrows != b.Hrows || a.B != b.B ||
            a.Bp != b.Bp || a.tks != b.tks || hs[j]->idx_hash != hs[k]->idx_hash ||
            hs[j]->idx_h != hs[k]->idx_h)
          continue;
        b.hs_hi = a.hs_hi;
        b.hs_lo = a.hs_lo;
        b.hs_shared = 1;
        break;
      }
    TDA_TRY(enqueue_mixed(mc->ring, mis, ris, hs, (double *)P.ws_fft.p, max_m, s));
    HIP_TRY(mc->ring.reserve(4096 + n_items * 16 + group_out.size() * 16));
  }
  // network sums per output array, in item order
  void *d_off, *d_grp, *d_outs, *d_Bs;
  HIP_TRY(mc->ring.push(part_off.data(), n_items * sizeof(int64_t), s, &d_off));
  HIP_TRY(mc->ring.push(group_of.data(), n_items * sizeof(int32_t), s, &d_grp));
  HIP_TRY(mc->ring.push(group_out.data(), group_out.size() * sizeof(double *), s, &d_outs));
  HIP_TRY(mc->ring.push(group_B.data(), group_B.size() * sizeof(int64_t), s, &d_Bs));
  HIP_TRY(launch_combine(partbuf, (const int64_t *)d_off, (const int32_t *)d_grp, n_items,
                         (double *const *)d_outs, (const int64_t *)d_Bs,
                         (int64_t)group_out.size(), max_B, s));
  HIP_TRY(mc->ring.seal(s));
  if (!capturing) HIP_TRY(hipEventRecord(mc->done, s));
  if (order_handles)
    for (int64_t k = 0; k < n_items; ++k) TDA_TRY(mark_done(items[k].h, s));
  return TDA_OK;
}
}  // namespace

// ---------------------------------------------------------------- plans and HIP graphs

struct tda_plan {
  MultiCtx *mc = nullptr;
  std::vector<tda_work> items;
  int32_t precision = TDA_PREC_FP64;
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" tda_status tda_plan_create(const tda_work *items, int64_t n_items, int32_t precision,
                                      tda_plan_t *out) {
  if (!out) return fail_with(TDA_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_items < 1 || !items || !items[0].h) return fail_with(TDA_EINVAL, "bad item list");
  tda_plan *p = new tda_plan();
  p->items.assign(items, items + n_items);
  p->precision = precision;
  p->device = items[0].h->device;
  p->mc = multi_ctx_create();
  DeviceGuard guard(p->device);
  hipStream_t s = nullptr;
  tda_status st = TDA_OK;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    st = fail_with(TDA_EHIP, "plan: stream creation failed");
  } else {
    HIP_TRY(hipDeviceSynchronize());
    st = multi_impl(p->mc, p->items.data(), nullptr, n_items, precision, s, false);
    if (st == TDA_OK && hipStreamSynchronize(s) != hipSuccess)
      st = fail_with(TDA_EHIP, "plan: first evaluation failed");
    (void)hipStreamDestroy(s);
  }
  if (st != TDA_OK) {
    multi_ctx_destroy(p->mc);
    delete p;
    return st;
  }
  *out = p;
  return TDA_OK;
}

extern "C" tda_status tda_plan_execute(tda_plan_t p, void *hip_stream, int32_t use_graph) {
  if (!p) return fail_with(TDA_EINVAL, "NULL plan");
  DeviceGuard guard(p->device);
  hipStream_t s = (hipStream_t)hip_stream;
  if (!p->exec && !use_graph)
    return multi_impl(p->mc, p->items.data(), nullptr, (int64_t)p->items.size(), p->precision,
                      s, false);
  if (!p->exec) {
    if (!s) return fail_with(TDA_EINVAL, "graph capture needs a non-default stream");
    // the graph replays copies out of its own descriptor slot, sized from the eager
    // evaluation of the same items
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(p->mc->ring.begin_graph(p->mc->ring.last_used));
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const tda_status st = multi_impl(p->mc, p->items.data(), nullptr, (int64_t)p->items.size(),
                                     p->precision, s, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    p->mc->ring.end_graph();
    if (st != TDA_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail_with(TDA_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    p->graph = g;
    HIP_TRY(hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(p->exec, s));
  return TDA_OK;
}

extern "C" tda_status tda_plan_destroy(tda_plan_t p) {
  if (!p) return TDA_OK;
  {
    DeviceGuard guard(p->device);
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    multi_ctx_destroy(p->mc);
  }
  delete p;
  return TDA_OK;
}

// ---------------------------------------------------------------- kernel timing

namespace {
struct TimingState {
  std::mutex mu;
  bool on = false;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::vector<tda_kernel_time> totals;
};
TimingState &timing() {
  static TimingState t;
  return t;
}
hipEvent_t pool_event(TimingState &t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
}  // namespace

namespace tda {
TimedScope::TimedScope(const char *n, hipStream_t s) : name(n), stream(s), slot(-1) {
  TimingState &t = timing();
  if (!t.on) return;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lk(t.mu);
  TimingState::Rec r{n, pool_event(t), pool_event(t)};
  (void)hipEventRecord(r.a, s);
  t.pending.push_back(r);
  slot = (int)t.pending.size() - 1;
}
TimedScope::~TimedScope() {
  if (slot < 0) return;
  TimingState &t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  if (slot < (int)t.pending.size()) (void)hipEventRecord(t.pending[slot].b, stream);
}
}  // namespace tda

extern "C" tda_status tda_timing_enable(int32_t on) {
  timing().on = on != 0;
  return TDA_OK;
}

extern "C" tda_status tda_timing_read(tda_kernel_time *out, int32_t max, int32_t *n,
                                      int32_t reset) {
  TimingState &t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  for (auto &r : t.pending) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    tda_kernel_time *slot = nullptr;
    for (auto &k : t.totals)
      if (r.name == k.name) slot = &k;
    if (!slot) {
      tda_kernel_time k{};
      snprintf(k.name, sizeof k.name, "%s", r.name.c_str());
      t.totals.push_back(k);
      slot = &t.totals.back();
    }
    slot->count += 1;
    slot->total_ms += ms;
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.pending.clear();
  const int32_t cnt = (int32_t)std::min<size_t>(t.totals.size(), max > 0 ? max : 0);
  for (int32_t k = 0; k < cnt; ++k) out[k] = t.totals[k];
  if (n) *n = (int32_t)t.totals.size();
  if (reset) t.totals.clear();
  return TDA_OK;
}

// ---------------------------------------------------------------- info / destroy / strings

extern "C" tda_status tda_info(tda_handle h, tda_info_t *info) {
  if (!h || !info) return fail_with(TDA_EINVAL, "NULL argument");
  info->n = h->N;
  info->n_eff = h->n_eff;
  info->n_pad = h->n_pad;
  info->n_segments = (int64_t)h->segs.size();
  info->logdet = h->logdet;
  info->fail_row = h->fail_row;
  info->fail_segment = h->fail_segment;
  info->factored = h->factored ? 1 : 0;
  info->precision = h->precision;
  info->data_set = h->data_ptr ? 1 : 0;
  info->device_bytes = h->held;
  return TDA_OK;
}

extern "C" tda_status tda_destroy(tda_handle h) {
  if (!h) return TDA_OK;
  {
    DeviceGuard guard(h->device);
    hipDeviceSynchronize();
    h->release_all();
    if (h->done) hipEventDestroy(h->done);
    h->ring.destroy();
  }
  delete h;
  return TDA_OK;
}

extern "C" const char *tda_status_str(tda_status s) {
  switch (s) {
    case TDA_OK: return "TDA_OK";
    case TDA_EINVAL: return "TDA_EINVAL: invalid argument";
    case TDA_ENOTSPD: return "TDA_ENOTSPD: covariance not positive definite";
    case TDA_ENOMEM: return "TDA_ENOMEM: out of device memory or budget";
    case TDA_ESTATE: return "TDA_ESTATE: call out of order";
    case TDA_ENODEV: return "TDA_ENODEV: no HIP device";
    case TDA_EHIP: return "TDA_EHIP: HIP runtime error";
    case TDA_EINTERNAL: return "TDA_EINTERNAL: internal error";
    case TDA_EAGAIN: return "TDA_EAGAIN: not admitted now, retry";
  }
  return "unknown status";
}

extern "C" const char *tda_last_error(void) { return g_err.c_str(); }

namespace {
void set_kernel_attributes() { tda::register_kernel_attributes(); }
}  // namespace
