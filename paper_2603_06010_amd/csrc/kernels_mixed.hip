// Mixed-precision kernels (gfx950): BF16 hi/lo split of the whitening operator
// W = L^-1 and of the templates, the two BF16x3 triangular products
//   w0 = W h           (row blocks of W, lower part)
//   y0 = W^T w0        (column blocks of W)
// with FP32 accumulation, the FP64 whitened-data cache, the circulant
// eigenvalues of each segment and the FP64 FFT refinement.
//
// BF16 matrix-core op (v_mfma_f32_32x32x16_bf16): D(32x32) += A(32x16) B(16x32);
// lane l supplies A[l%32][8(l/32)+e] and B[8(l/32)+e][l%32] (e = 0..7) and holds
// D[8(j/4) + 4(l/32) + j%4][l%32] in register j (j = 0..15).
//
// Fragment layout F(M) of a matrix M with rows in tiles of 32 and columns in
// k-steps of 16: fragment (tile, kstep) is 64 lanes x 8 bf16, lane l holding
// M[32 tile + l%32][16 kstep + 8(l/32) + e].  A fragment of F(M) is the A operand
// for rows of M; a fragment of F(M^T) is the B operand for columns of M.
#include <math.h>

#include "tda_internal.h"

namespace tda {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f16v mfma_bf16(bf8 a, bf8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// round-to-nearest-even FP32 -> BF16 bits (NaN kept NaN): the hardware conversion
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// x ~ hi + lo with hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split2(double x, uint16_t &hi, uint16_t &lo) {
  hi = bf16_bits((float)x);
  lo = bf16_bits((float)(x - (double)bf16_float(hi)));
}
__device__ __forceinline__ void split2f(float x, uint16_t &hi, uint16_t &lo) {
  hi = bf16_bits(x);
  lo = bf16_bits(x - bf16_float(hi));
}

// Fragment load through a global-address-space pointer (a global_load, not a flat load
// that would also count against the LDS counter); every operand lives in device memory.
typedef __attribute__((address_space(1))) const bf8 gbf8;
__device__ __forceinline__ bf8 load_frag(const uint16_t *p) {
  return *(gbf8 *)(p);
}

// Device-memory views for the transform kernels: accesses through them compile to
// global loads and stores.  Pointers read out of a work item are generic, and flat accesses
// through them also count against the LDS counter, so each wait for an LDS read issued
// behind one would wait for device memory too.
template <class T> using gmem = __attribute__((address_space(1))) T;
template <class T> __device__ __forceinline__ gmem<T> *gp(T *p) { return (gmem<T> *)p; }
// Values that are the same in every lane, moved to scalar registers: pointers and sizes of a
// work item are uniform, but read through a reference argument of a called function the
// compiler cannot tell and holds each in vector registers.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
template <class T> __device__ __forceinline__ T *uni(T *p) {
  const uint64_t u = (uint64_t)p;
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (T *)(lo | (hi << 32));
}
// a uniform device-memory view
template <class T> __device__ __forceinline__ gmem<T> *gpu(T *p) { return uni(gp(p)); }
// complex doubles in device memory are read and written as a plain vector type (the HIP
// vector class has no address-space-qualified copy operations)
typedef double dv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 from_dv2(dv2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ dv2 to_dv2(double2 v) {
  dv2 r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

// ---------------------------------------------------------------- split fragment layout
// The products read templates and residuals as BF16 hi/lo in the layout [Bp/32][tks][64][8]:
// per tile of 32 templates and k-step of 16 padded rows, 64 lanes of 8 consecutive rows,
// lane = template mod 32 for rows 0..7 of the step and + 32 for rows 8..15.
__device__ __forceinline__ int64_t frag_col(int64_t b, int64_t tks) {
  return ((b >> 5) * tks * 64 + (b & 31)) * 8;  // template b's row 0
}
__device__ __forceinline__ int64_t frag_row(int64_t r) {
  return ((r >> 4) << 9) + (((r >> 3) & 1) << 8) + (r & 7);
}

// The refinement writes the residual e = h - C y0 of template b straight into that layout,
// split (what the template split does for h), for the correction product.
struct EsOut {
  gmem<uint16_t> *hi, *lo;
  __device__ __forceinline__ EsOut(uint16_t *es_hi, uint16_t *es_lo, int64_t tks, int64_t b) {
    const int64_t o = frag_col(b, tks);
    hi = gpu(es_hi + o);
    lo = gpu(es_lo + o);
  }
  __device__ __forceinline__ void put(int32_t r, double v) const {
    uint16_t h, l;
    split2(v, h, l);
    const int64_t o = frag_row(r);
    hi[o] = h;
    lo[o] = l;
  }
  // rows r[0], r[1] (-1: none); one 4-byte store per part when they are r, r + 1 with r even
  __device__ __forceinline__ void pair(const int32_t (&r)[2], double v0, double v1) const {
    if (r[0] >= 0 && r[1] == r[0] + 1 && !(r[0] & 1)) {
      uint16_t h0, l0, h1, l1;
      split2(v0, h0, l0);
      split2(v1, h1, l1);
      const int64_t o = frag_row(r[0]);
      *(gmem<uint32_t> *)(hi + o) = (uint32_t)h0 | ((uint32_t)h1 << 16);
      *(gmem<uint32_t> *)(lo + o) = (uint32_t)l0 | ((uint32_t)l1 << 16);
    } else {
      if (r[0] >= 0) put(r[0], v0);
      if (r[1] >= 0) put(r[1], v1);
    }
  }
};

// ---------------------------------------------------------------- W64 access
// W = L^-1 in FP64, compact column tiles of 32 columns: tile ct holds rows
// [rb[ct], segment end) at w64[off[ct] + (r - rb[ct]) * 32 + (c % 32)].
__device__ __forceinline__ double w64_at(const double *w64, const int64_t *off, const int32_t *rb,
                                         int64_t r, int64_t c) {
  const int64_t ct = c >> 5;
  if (r < c) return 0.0;
  return w64[off[ct] + (r - rb[ct]) * 32 + (c & 31)];
}

// grid: (chunks, nblk, 2); z = 0 builds F(W) row block i, z = 1 builds F(W^T) column block i.
__global__ void k_split_w(const double *__restrict__ w64, const int64_t *__restrict__ off,
                          const int32_t *__restrict__ rb, const int32_t *__restrict__ blk_first,
                          const int32_t *__restrict__ blk_last, uint16_t *__restrict__ wa_hi,
                          uint16_t *__restrict__ wa_lo, const int64_t *__restrict__ wa_off,
                          uint16_t *__restrict__ wb_hi, uint16_t *__restrict__ wb_lo,
                          const int64_t *__restrict__ wb_off) {
  const int i = blockIdx.y;
  const bool transposed = blockIdx.z == 1;
  const int64_t kbeg = transposed ? (int64_t)i * TB : (int64_t)blk_first[i] * TB;
  const int64_t kend = transposed ? (int64_t)(blk_last[i] + 1) * TB : (int64_t)(i + 1) * TB;
  const int64_t nks = (kend - kbeg) / 16;
  const int64_t chunk = (int64_t)blockIdx.x * 256 + threadIdx.x;  // (ks, rt, lane)
  if (chunk >= nks * 8 * 64) return;
  const int lane = (int)(chunk & 63), rt = (int)((chunk >> 6) & 7);
  const int64_t ks = chunk >> 9;
  const int64_t m_row = (int64_t)i * TB + 32 * rt + (lane & 31);      // row of M
  const int64_t k0 = kbeg + 16 * ks + 8 * (lane >> 5);                // first column of M
  uint16_t hi[8], lo[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const double v = transposed ? w64_at(w64, off, rb, k0 + e, m_row)   // M = W^T
                                : w64_at(w64, off, rb, m_row, k0 + e);  // M = W
    split2(v, hi[e], lo[e]);
  }
  const int64_t dst = ((transposed ? wb_off[i] : wa_off[i]) + chunk * 8);
  uint16_t *H = transposed ? wb_hi : wa_hi;
  uint16_t *L = transposed ? wb_lo : wa_lo;
  uint4 vh, vl;
  vh.x = hi[0] | ((uint32_t)hi[1] << 16); vh.y = hi[2] | ((uint32_t)hi[3] << 16);
  vh.z = hi[4] | ((uint32_t)hi[5] << 16); vh.w = hi[6] | ((uint32_t)hi[7] << 16);
  vl.x = lo[0] | ((uint32_t)lo[1] << 16); vl.y = lo[2] | ((uint32_t)lo[3] << 16);
  vl.z = lo[4] | ((uint32_t)lo[5] << 16); vl.w = lo[6] | ((uint32_t)lo[7] << 16);
  *reinterpret_cast<uint4 *>(H + dst) = vh;
  *reinterpret_cast<uint4 *>(L + dst) = vl;
}

hipError_t launch_split_w(const double *w64, const int64_t *w64_off, const int32_t *w64_rb,
                          const int32_t *blk_first, const int32_t *blk_last, int32_t nblk,
                          uint16_t *wa_hi, uint16_t *wa_lo, const int64_t *wa_off,
                          uint16_t *wb_hi, uint16_t *wb_lo, const int64_t *wb_off,
                          int64_t max_k, int64_t unused, hipStream_t s) {
  (void)unused;
  const int64_t max_chunks = (max_k / 16) * 8 * 64;
  dim3 grid((unsigned)((max_chunks + 255) / 256), (unsigned)nblk, 2);
  hipLaunchKernelGGL(k_split_w, grid, dim3(256), 0, s, w64, w64_off, w64_rb, blk_first, blk_last,
                     wa_hi, wa_lo, wa_off, wb_hi, wb_lo, wb_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------- whitened data (FP64)
// dbar = W d on retained rows, y_d = W^T dbar = C^-1 d, q_dd = dbar^T dbar (Sec. III.A:
// the whitened data vector is computed once and cached).  The cache is keyed by a
// fingerprint of the retained samples of d, taken on the device by every evaluation
// (k_data_check): the three whitening kernels run only when it differs from the cached
// one (chk->stale), so an in-place update of d, or new data at the cached address, is
// picked up without a host round trip.

// splitmix64 finaliser (Steele, Lea and Flood, OOPSLA 2014): a bijective 64-bit mixer.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// One workgroup.  fp = sum over retained rows r of mix64(bits(d[idx[r]]) + mix64(r)) mod
// 2^64 (order-free, so reproducible).  Then: equal to the cached fingerprint -> not stale,
// chk->qdd = the cached q_dd; else, if the handle can whiten (its FP64 operator is held)
// -> stale (the whitening kernels recompute and k_qdd_and_scatter stores the fingerprint);
// else (compact handle) -> not stale and chk->qdd = NaN, so every result of the call is NaN.
__global__ __launch_bounds__(1024) void k_data_check(const double *__restrict__ d,
                                                     const int32_t *__restrict__ idx,
                                                     int32_t n_pad, DataCache *__restrict__ cache,
                                                     DataCheck *__restrict__ chk,
                                                     int32_t can_whiten, int32_t force) {
  __shared__ uint64_t part[1024];
  // rows in rounds of 16 per thread, every load of a round issued before the hashing (the
  // sum does not depend on the order)
  constexpr int U = 16;
  uint64_t acc = 0;
  for (int32_t r0 = 0; r0 < n_pad; r0 += 1024 * U) {
    int32_t p[U];
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t r = r0 + (int32_t)threadIdx.x + 1024 * u;
      p[u] = r < n_pad ? idx[r] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = p[u] >= 0 ? d[p[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t r = r0 + (int32_t)threadIdx.x + 1024 * u;
      if (p[u] >= 0) acc += mix64((uint64_t)__double_as_longlong(v[u]) + mix64((uint64_t)r));
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint64_t fp = part[0];
    chk->fp = fp;
    const bool match = !force && cache->valid == 1 && cache->fp == fp;
    if (match) {
      chk->stale = 0;
      chk->qdd = cache->qdd;
    } else if (can_whiten) {
      chk->stale = 1;
    } else {
      chk->stale = 0;
      chk->qdd = __builtin_nan("");
    }
  }
}

// d-bar = W d over the padded rows.  A workgroup takes DB_ROWS consecutive rows (inside one
// 256-row block, so one segment) as 8 row groups x 32 columns of a column tile: a row's 32
// entries in a tile are contiguous, so each row group reads 256 contiguous bytes per row.
// It sums over the segment's tiles up to its last row, then over the 32 columns in the
// wave (fixed order).
constexpr int DB_ROWS = 32;
__global__ __launch_bounds__(256) void k_dbar(const double *__restrict__ w64,
                                              const int64_t *__restrict__ off,
                                              const int32_t *__restrict__ rb,
                                              const int32_t *__restrict__ blk_first,
                                              const int32_t *__restrict__ idx,
                                              const double *__restrict__ d,
                                              double *__restrict__ dbar,
                                              const DataCheck *__restrict__ chk) {
  if (!chk->stale) return;
  constexpr int NR = DB_ROWS / 8;
  const int cc = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * DB_ROWS;
  const int64_t ct_beg = (int64_t)blk_first[r0 / TB] * (TB / 32);
  const int64_t ct_end = (r0 + DB_ROWS - 1) / 32;  // the tile of the last row's diagonal
  double acc[NR];
#pragma unroll
  for (int u = 0; u < NR; ++u) acc[u] = 0.0;
#pragma unroll 4
  for (int64_t ct = ct_beg; ct <= ct_end; ++ct) {
    const int64_t c = ct * 32 + cc;
    const int32_t p = idx[c];
    const double dv = p >= 0 ? d[p] : 0.0;
    const double *wt = w64 + off[ct] + cc;
    const int64_t rbt = rb[ct];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int64_t r = r0 + g + 8 * u;
      if (r >= c) acc[u] += wt[(r - rbt) * 32] * dv;
    }
  }
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    double v = acc[u];
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
    if (cc == 0) dbar[r0 + g + 8 * u] = v;
  }
}

// y_d = W^T d-bar: a workgroup per column tile, 8 row groups x 32 columns (256 contiguous
// bytes per row), eight independent partial sums per thread over rows r = g + 8 k, then the
// row groups in LDS (fixed order).
__global__ void k_yd(const double *__restrict__ w64, const int64_t *__restrict__ off,
                     const int32_t *__restrict__ rb, const int32_t *__restrict__ blk_last,
                     const double *__restrict__ dbar, double *__restrict__ yd,
                     const DataCheck *__restrict__ chk) {
  if (!chk->stale) return;
  __shared__ double part[8][32];
  const int ct = blockIdx.x;
  const int cc = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int64_t c = (int64_t)ct * 32 + cc;
  const int64_t r_end = (int64_t)(blk_last[c / TB] + 1) * TB;
  const int64_t rbt = rb[ct];
  const double *wt = w64 + off[ct] + cc;
  auto term = [&](int64_t r) { return r >= c ? wt[(r - rbt) * 32] * dbar[r] : 0.0; };
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t r = rbt + g;
  for (; r + 56 < r_end; r += 64) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += term(r + 8 * k);
  }
  for (; r < r_end; r += 8) a[0] += term(r);
  part[g][cc] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  if (g == 0) {
    double s = 0.0;
    for (int k = 0; k < 8; ++k) s += part[k][cc];
    yd[c] = s;
  }
}

// q_dd, and y_d scattered to sample positions (0 at excluded samples).  Every position is
// written once with its final value, so a concurrent evaluation on another stream that
// reads the cache never sees a transient value; the fingerprint is published last, after
// a device-scope fence, so a reader that sees it also sees the values it keys.
__global__ void k_qdd_and_scatter(const double *__restrict__ dbar, const double *__restrict__ yd,
                                  const int32_t *__restrict__ pos2row, int32_t n_pad, int64_t N,
                                  double *__restrict__ yd_pos, DataCache *__restrict__ cache,
                                  DataCheck *__restrict__ chk) {
  if (!chk->stale) return;
  __shared__ double part[256];
  for (int64_t j = threadIdx.x; j < N; j += 256) {
    const int32_t r = pos2row[j];
    yd_pos[j] = r >= 0 ? yd[r] : 0.0;
  }
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n_pad; r += 256) s += dbar[r] * dbar[r];
  part[threadIdx.x] = s;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 256; ++k) t += part[k];
    chk->qdd = t;
    cache->qdd = t;
    __threadfence();
    cache->fp = chk->fp;
    cache->valid = 1;
  }
}

hipError_t launch_data_check(const double *d, const int32_t *idx, int32_t n_pad, DataCache *cache,
                             DataCheck *chk, int32_t can_whiten, int32_t force, hipStream_t s) {
  hipLaunchKernelGGL(k_data_check, dim3(1), dim3(1024), 0, s, d, idx, n_pad, cache, chk,
                     can_whiten, force);
  return hipGetLastError();
}

hipError_t launch_data_whiten(const double *w64, const int64_t *w64_off, const int32_t *w64_rb,
                              const int32_t *blk_first, const int32_t *blk_last, const int32_t *idx,
                              const int32_t *pos2row, int32_t n_pad, int64_t N, const double *d,
                              double *dbar, double *yd, double *yd_pos, DataCache *cache,
                              DataCheck *chk, hipStream_t s) {
  hipLaunchKernelGGL(k_dbar, dim3((unsigned)(n_pad / DB_ROWS)), dim3(256), 0, s, w64, w64_off,
                     w64_rb, blk_first, idx, d, dbar, (const DataCheck *)chk);
  hipLaunchKernelGGL(k_yd, dim3((unsigned)(n_pad / 32)), dim3(256), 0, s, w64, w64_off, w64_rb,
                     blk_last, dbar, yd, (const DataCheck *)chk);
  hipLaunchKernelGGL(k_qdd_and_scatter, dim3(1), dim3(256), 0, s, dbar, yd, pos2row, n_pad, N,
                     yd_pos, cache, chk);
  return hipGetLastError();
}

// ---------------------------------------------------------------- circulant eigenvalues
// Circulant embedding of the segment's Toeplitz block (eq:toeplitz_fft), m >= 2 length:
// c_j = acf[j] (j < length), c_{m-j} = acf[j] (1 <= j < length), 0 otherwise;
// lambda_k = sum_j c_j cos(2 pi j k / m) = acf[0] + 2 sum_{j>=1} acf[j] cos(2 pi j k / m).
__global__ void k_twiddles(int64_t m, double *__restrict__ tw) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= m) return;
  double sn, cs;
  sincospi(2.0 * (double)r / (double)m, &sn, &cs);
  tw[2 * r] = cs;
  tw[2 * r + 1] = sn;
}

__global__ void k_lambda(const double *__restrict__ acf, int64_t length, int64_t m,
                         const double *__restrict__ tw, double *__restrict__ lam) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= m) return;
  double s = 0.0;
  int64_t r = 0;
  for (int64_t j = 1; j < length; ++j) {
    r += k;
    if (r >= m) r -= m;  // r = j k mod m (k < m)
    s += acf[j] * tw[2 * r];
  }
  lam[k] = acf[0] + 2.0 * s;
}

// Pass twiddles of the in-LDS h-point DFT (h = 2^LH): for pass p >= 1 with sub-transform
// length Ns and radix R, entry [k][q-1] = w_{Ns R}^{q k} (k < Ns, q = 1 .. R-1), so that
// the R - 1 twiddles of one sub-transform are contiguous.
__global__ void k_pass_twiddles(int LH, double *__restrict__ ptw) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= rl_tw_size(LH)) return;
  int p = 1;
  while (p + 1 < rl_npass(LH) && i >= rl_off(LH, p + 1)) ++p;
  const int ns = 1 << rl_lns(LH, p), r = 1 << rl_L(LH, p);
  const int u = i - rl_off(LH, p), q = u % (r - 1) + 1, k = u / (r - 1);
  const int len = ns * r, e = (q * k) % len;
  double sn, cs;
  sincospi(2.0 * (double)e / (double)len, &sn, &cs);
  ptw[2 * i] = cs;
  ptw[2 * i + 1] = -sn;
}

hipError_t launch_lambda(const double *acf, int64_t length, int64_t m, double *tw, double *lam,
                         double *ptw, hipStream_t s) {
  const unsigned g = (unsigned)((m + 255) / 256);
  hipLaunchKernelGGL(k_twiddles, dim3(g), dim3(256), 0, s, m, tw);
  if (lam) hipLaunchKernelGGL(k_lambda, dim3(g), dim3(256), 0, s, acf, length, m, tw, lam);
  if (ptw && m >= 16 && m <= RL_MAX_M_QUAD) {
    int lm = 0;
    while (((int64_t)1 << lm) < m) ++lm;
    // the m/4-point DFT, or its halves or quarters beyond the LDS array
    const int lh = lm - 2 <= RL_LHMAX ? lm - 2 : RL_LHMAX;
    const int n = rl_tw_size(lh);
    if (n > 0) hipLaunchKernelGGL(k_pass_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, lh, ptw);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- template split
// F(Hs): rows = templates (padded to Bp), K = padded sample rows; Hs[b][p] = h_b[idx[p]].
// grid (chunks of the largest item, items); each item has (Bp/32) (n_pad/16) 64 chunks of
// 8 rows of one template
__global__ void k_split_h(const MixItem *__restrict__ items) {
  const MixItem &it = items[blockIdx.y];
  const int64_t nks = it.n_pad / 16;
  const int64_t chunks = (int64_t)(it.Bp / 32) * nks * 64;
  const int64_t chunk = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (chunk >= chunks || it.B == 0 || it.hs_shared) return;
  const int lane = (int)(chunk & 63);
  const int64_t ks = (chunk >> 6) % nks;
  const int64_t tt = (chunk >> 6) / nks;
  const int64_t dst = ((tt * it.tks + ks) * 64 + lane) * 8;
  const int64_t b = 32 * tt + (lane & 31);
  const int64_t p0 = 16 * ks + 8 * (lane >> 5);
  // the eight rows' samples, gathered through idx (read as two 16-byte loads); rows that
  // are eight consecutive samples at a 16-byte boundary are read as four 16-byte loads
  const int4 *ip = reinterpret_cast<const int4 *>(it.idx + p0);
  const int4 i0 = ip[0], i1 = ip[1];
  const int32_t pr[8] = {i0.x, i0.y, i0.z, i0.w, i1.x, i1.y, i1.z, i1.w};
  const double *row = b < it.B ? template_row(it, b) : nullptr;
  double v[8];
  if (row && pr[0] >= 0 && pr[7] == pr[0] + 7 && !(((uintptr_t)(row + pr[0])) & 15)) {
    const double2 *src = reinterpret_cast<const double2 *>(row + pr[0]);
    const double2 u0 = src[0], u1 = src[1], u2 = src[2], u3 = src[3];
    v[0] = u0.x; v[1] = u0.y; v[2] = u1.x; v[3] = u1.y;
    v[4] = u2.x; v[5] = u2.y; v[6] = u3.x; v[7] = u3.y;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (row && pr[e] >= 0) ? row[pr[e]] : 0.0;
  }
  uint16_t hi[8], lo[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) split2(v[e], hi[e], lo[e]);
  uint4 vh, vl;
  vh.x = hi[0] | ((uint32_t)hi[1] << 16); vh.y = hi[2] | ((uint32_t)hi[3] << 16);
  vh.z = hi[4] | ((uint32_t)hi[5] << 16); vh.w = hi[6] | ((uint32_t)hi[7] << 16);
  vl.x = lo[0] | ((uint32_t)lo[1] << 16); vl.y = lo[2] | ((uint32_t)lo[3] << 16);
  vl.z = lo[4] | ((uint32_t)lo[5] << 16); vl.w = lo[6] | ((uint32_t)lo[7] << 16);
  *reinterpret_cast<uint4 *>(it.hs_hi + dst) = vh;
  *reinterpret_cast<uint4 *>(it.hs_lo + dst) = vl;
}

hipError_t launch_split_h(const MixItem *items, int32_t n_items, int64_t max_chunks,
                          hipStream_t s) {
  if (n_items <= 0 || max_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_h, dim3((unsigned)((max_chunks + 255) / 256), (unsigned)n_items),
                     dim3(256), 0, s, items);
  return hipGetLastError();
}

// ---------------------------------------------------------------- BF16x3 products
// A workgroup computes a tile of D = A B over K = 16 nks; A and B are given as fragment
// arrays: A tile t (32 rows) at k-step ks is at A + t s_tile + ks s_ks.  Every product is
// hi*hi + hi*lo + lo*hi with FP32 accumulation.  Variants (picked per shape by the
// autotuner):
//   1: 4 waves, wave tile 4 A x 4 B tiles (128 x 128), workgroup 256 x 256, loads one
//      k-step ahead straight into registers; one wave per SIMD (accumulators in AGPRs).
//   2: 4 waves, wave tile 4 x 2, workgroup 256 x 128 (half a template group); two
//      workgroups per CU, so two waves per SIMD hide each other's latency.
//   4: as 1 with three register stages (loads two k-steps ahead).
//   5: 8 waves (two per SIMD), wave tile 4 x 2, workgroup 256 x 256.  Each k-step's 32
//      fragments go once per workgroup from memory into a 4-stage LDS ring (direct
//      global -> LDS loads, three k-steps ahead), and every wave reads its 12 fragments of
//      the next k-step from LDS while its matrix-core ops work on the current one.  The
//      register variants fetch each fragment twice per workgroup (two waves share every A
//      and every B tile), which keeps the vector-memory path busier than the matrix cores.
struct FragSrc {
  const uint16_t *hi, *lo;
  int64_t s_tile, s_ks;  // element strides between tiles and between k-steps
};

constexpr int FRAG = 512;  // bf16 elements per fragment (64 lanes x 8)

// Layout of variant V: waves per workgroup, B tiles per wave, whether a workgroup covers
// a whole group of 256 templates (else half, chosen by the work entry's `sub`), register
// stages, workgroups per CU, waves per SIMD, LDS stages, and the wave's first A and B tile.
template <int V>
struct PL {
  static constexpr int NW = V == 5 ? 8 : 4;
  static constexpr int WB = V == 2 || V == 5 ? 2 : 4;
  static constexpr bool FULL = V != 2;
  static constexpr int RST = V == 4 ? 3 : 2;
  static constexpr int OCC = V == 2 ? 2 : 1;
  static constexpr int WPS = NW * OCC / 4;
  static constexpr int LDS_STAGES = V == 5 ? 4 : 0;
  __device__ static int ta(int w) { return NW == 8 ? 4 * (w >> 2) : 4 * (w >> 1); }
  __device__ static int tb(int w) { return NW == 8 ? 2 * (w & 3) : WB * (w & 1); }
  static constexpr size_t lds_bytes() { return (size_t)LDS_STAGES * 32 * FRAG * 2; }
};

template <int WB>
struct Step {
  bf8 ah[4], al[4], bh[WB], bl[WB];
};

// NPROD = 3: hi*hi + hi*lo + lo*hi; NPROD = 1: hi*hi only (lo parts not loaded)
// Issued in the order mma_step consumes them: A hi and B hi (first pass), B lo, A lo.
template <int NPROD, int WB>
__device__ __forceinline__ void load_step(const FragSrc &A, const FragSrc &B, int ta, int tb,
                                          int64_t ks, int lane, Step<WB> &st) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
    st.ah[a] = load_frag(A.hi + (int64_t)(ta + a) * A.s_tile + ks * A.s_ks + lane * 8);
#pragma unroll
  for (int b = 0; b < WB; ++b)
    st.bh[b] = load_frag(B.hi + (int64_t)(tb + b) * B.s_tile + ks * B.s_ks + lane * 8);
  if (NPROD == 3) {
#pragma unroll
    for (int b = 0; b < WB; ++b)
      st.bl[b] = load_frag(B.lo + (int64_t)(tb + b) * B.s_tile + ks * B.s_ks + lane * 8);
#pragma unroll
    for (int a = 0; a < 4; ++a)
      st.al[a] = load_frag(A.lo + (int64_t)(ta + a) * A.s_tile + ks * A.s_ks + lane * 8);
  }
}

template <int NPROD, int WB>
__device__ __forceinline__ void mma_step(const Step<WB> &st, f16v (&acc)[4][WB]) {
  // separate passes so consecutive matrix-core ops use independent accumulators
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b) acc[a][b] = mfma_bf16(st.ah[a], st.bh[b], acc[a][b]);
  if (NPROD == 3) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < WB; ++b) acc[a][b] = mfma_bf16(st.ah[a], st.bl[b], acc[a][b]);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < WB; ++b) acc[a][b] = mfma_bf16(st.al[a], st.bh[b], acc[a][b]);
  }
}

template <int WB>
__device__ __forceinline__ void zero_acc(f16v (&acc)[4][WB]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b) acc[a][b] = f16v{};
}

// NST register stages, loads issued NST - 1 k-steps
// ahead.  The scheduling barriers keep each k-step's loads ahead of the matrix-core ops
// before them, and the loop body has no branch (loads past the end are clamped to the
// last k-step), so the compiler's wait counts leave the later stages in flight.
template <int NPROD, int WB, int NST>
__device__ __forceinline__ void gemm3(const FragSrc &A, const FragSrc &B, int ta, int tb,
                                      int64_t nks, int lane, f16v (&acc)[4][WB]) {
  zero_acc<WB>(acc);
  if (nks <= 0) return;
  Step<WB> st[NST];
#pragma unroll
  for (int p = 0; p < NST - 1; ++p)
    load_step<NPROD, WB>(A, B, ta, tb, p < nks ? p : nks - 1, lane, st[p]);
  // loads of a later k-step are spread through this k-step's matrix-core ops
  constexpr int NL = (NPROD == 3 ? 2 : 1) * (4 + WB), NM = NPROD * 4 * WB;
  int64_t ks = 0;
  for (; ks + NST <= nks; ks += NST) {
#pragma unroll
    for (int u = 0; u < NST; ++u) {
      const int64_t kn = ks + u + NST - 1;
      load_step<NPROD, WB>(A, B, ta, tb, kn < nks ? kn : nks - 1, lane, st[(u + NST - 1) % NST]);
      mma_step<NPROD, WB>(st[u], acc);
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);        // one global load
        __builtin_amdgcn_sched_group_barrier(0x008, NM / NL, 0);  // then matrix-core ops
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // remaining nks mod NST steps sit in the first stages
  const int64_t rem = nks - ks;
#pragma unroll
  for (int u = 0; u < NST - 1; ++u)
    if (u < rem) mma_step<NPROD, WB>(st[u], acc);
}

// LDS path (variant 5).  A stage holds one k-step's 32 fragments: A hi tiles 0-7, A lo
// 0-7, B hi 0-7, B lo 0-7 of the workgroup's window; wave w copies fragments 4w .. 4w + 3
// (one quarter of one of the four arrays).  Loads past the last k-step are clamped to it
// (their stage is never read), so every k-step issues the same four copies and the wait
// counts are constants.  The barrier at k-step t follows the wave's wait for its copies of
// stage t + 1: after it stage t + 1 is complete for every wave and stage t - 1, which the
// new copies overwrite, has been read by all of them.
typedef __attribute__((address_space(3))) void lds_void_t;

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int WB>
__device__ __forceinline__ void lds_read_step(const char *stage, int ta, int tb, int lane,
                                              Step<WB> &st) {
  const bf8 *S = (const bf8 *)stage;
#pragma unroll
  for (int a = 0; a < 4; ++a) st.ah[a] = S[(ta + a) * 64 + lane];
#pragma unroll
  for (int b = 0; b < WB; ++b) st.bh[b] = S[(16 + tb + b) * 64 + lane];
#pragma unroll
  for (int b = 0; b < WB; ++b) st.bl[b] = S[(24 + tb + b) * 64 + lane];
#pragma unroll
  for (int a = 0; a < 4; ++a) st.al[a] = S[(8 + ta + a) * 64 + lane];
}

template <int NPROD, int V>
__device__ __forceinline__ void gemm_lds(const FragSrc &A, const FragSrc &B, int64_t nks, int tid,
                                         f16v (&acc)[4][PL<V>::WB], char *smem) {
  using L = PL<V>;
  constexpr int NS = L::LDS_STAGES, SB = 32 * FRAG * 2;
  constexpr int FPW = 32 / L::NW;  // fragments each wave copies per stage
  static_assert(L::NW == 8 && NS >= 3, "LDS path: 8 waves, at least 3 stages");
  const int lane = tid & 63, w = tid >> 6;
  const int ta = L::ta(w), tb = L::tb(w);
  // this wave's copies: fragments FPW w .. FPW w + FPW - 1 of the stage, which lie in one
  // array (A hi, A lo, B hi, B lo: 8 tiles each)
  const int f0 = FPW * w, arr = f0 >> 3;
  const bool isA = arr < 2;
  const uint16_t *src = arr == 0 ? A.hi : arr == 1 ? A.lo : arr == 2 ? B.hi : B.lo;
  const int64_t s_tile = isA ? A.s_tile : B.s_tile, s_ks = isA ? A.s_ks : B.s_ks;
  const uint16_t *gp = src + (f0 & 7) * s_tile + lane * 8;
  char *const dst0 = smem + f0 * 1024;
  auto issue = [&](int64_t ks, int slot) __attribute__((always_inline)) {
    const uint16_t *q = gp + (ks < nks ? ks : nks - 1) * s_ks;
#pragma unroll
    for (int u = 0; u < FPW; ++u)
      __builtin_amdgcn_global_load_lds((const void *)(q + u * s_tile),
                                       (lds_void_t *)(dst0 + slot * SB + u * 1024), 16, 0, 0);
  };
  auto next_slot = [](int sl) __attribute__((always_inline)) { return sl + 1 == NS ? 0 : sl + 1; };
  zero_acc<L::WB>(acc);
  if (nks <= 0) return;
#pragma unroll
  for (int p = 0; p < NS - 1; ++p) issue(p, p);
  wait_vmcnt<FPW * (NS - 2)>();
  __builtin_amdgcn_s_barrier();
  Step<L::WB> r0, r1;
  lds_read_step<L::WB>(smem, ta, tb, lane, r0);
  // one k-step: wait for stage t + 1, barrier, copies for stage t + NS - 1 (into the slot
  // of stage t - 1), LDS reads of stage t + 1 spread through the matrix-core ops of
  // stage t.  s1 is the slot of stage t + 1.
  auto kstep = [&](int64_t t, int s1, const Step<L::WB> &cur, Step<L::WB> &nxt) __attribute__((always_inline)) {
    wait_vmcnt<FPW * (NS - 3)>();
    __builtin_amdgcn_s_barrier();
    issue(t + NS - 1, s1 == 0 ? NS - 2 : s1 == 1 ? NS - 1 : s1 - 2);
    lds_read_step<L::WB>(smem + s1 * SB, ta, tb, lane, nxt);
    mma_step<NPROD, L::WB>(cur, acc);
    // matrix-core ops first: their operands were read a k-step ago, so the wait for them
    // does not also wait for the reads of the next stage
    constexpr int NR = 4 + 2 * L::WB + 4, NM = NPROD * 4 * L::WB;
    __builtin_amdgcn_sched_group_barrier(0x020, FPW, 0);      // the copies
    __builtin_amdgcn_sched_group_barrier(0x008, NM / NR, 0);  // matrix-core ops
#pragma unroll
    for (int q = 0; q < NR - 1; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);        // one LDS read
      __builtin_amdgcn_sched_group_barrier(0x008, NM / NR, 0);  // then matrix-core ops
    }
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    __builtin_amdgcn_sched_barrier(0);
  };
  int64_t t = 0;
  int s1 = 1;  // slot of stage t + 1
  for (; t + 2 <= nks; t += 2) {
    kstep(t, s1, r0, r1);
    s1 = next_slot(s1);
    kstep(t + 1, s1, r1, r0);
    s1 = next_slot(s1);
  }
  if (t < nks) mma_step<NPROD, L::WB>(r0, acc);
  // no copy may still be landing in LDS when the workgroup reuses or releases it
  wait_vmcnt<0>();
  __builtin_amdgcn_s_barrier();
}

template <int NPROD, int V>
__device__ __forceinline__ void gemm3_v(const FragSrc &A, const FragSrc &B, int64_t nks, int tid,
                                        f16v (&acc)[4][PL<V>::WB]) {
  using L = PL<V>;
  if constexpr (L::LDS_STAGES > 0) {
    extern __shared__ char gp_smem[];
    gemm_lds<NPROD, V>(A, B, nks, tid, acc, gp_smem);
  } else {
    const int w = tid >> 6;
    gemm3<NPROD, L::WB, L::RST>(A, B, L::ta(w), L::tb(w), nks, tid & 63, acc);
  }
}

// The thread index behind a barrier the compiler cannot see through.  Each block of a pair
// derives its lane-dependent addresses from its own read, so none are kept live across the
// other block's product, where they would spill registers.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Work entries (item, block, group of 256 templates, sub): half-group variants take the
// half `sub`; full-group variants cover both halves at sub = 0 and skip sub = 1.
//
// Block pairs.  In a segment of nb blocks the products over block l (local index) run
// over l + 1 blocks of K (forward, correction) or nb - l (backward), so a workgroup per
// block would see lengths from 1 to nb and start at staggered times, which defeats the
// L2 sharing of the work order.  A workgroup instead takes block l and its partner
// nb - 1 - l (the middle block of an odd segment alone): every pair spans nb + 1 blocks of
// K.  The second block's K range is walked in the opposite direction, which lines the
// walks up in time: at a given k-step of their run, all workgroups of a segment read one
// of just two template k-steps, whichever pair they hold.  The entry names the first
// block of the pair (the lower index); `ph` selects the first (0) or second (1) block.
__device__ __forceinline__ int pair_blocks(const MixItem &it, int first) {
  return it.blk_first[first] + it.blk_last[first] - first != first ? 2 : 1;
}

// w0 = W h: rows of row block i (A = F(W)), templates of the group (B = F(Hs)); w0 is
// written in F(w0^T).  The first block of the pair walks K upwards, its partner downwards.
template <int V, int ph>
__device__ __forceinline__ void fwd_block(const MixItem *items, const int4 *work) {
  using L = PL<V>;
  const int4 wk = work[blockIdx.x];
  const MixItem &it = items[wk.x];
  const int tid = opaque_tid();
  const int bf = it.blk_first[wk.y];
  const int i = ph ? bf + it.blk_last[wk.y] - wk.y : wk.y;
  const int64_t ks0 = (int64_t)bf * (TB / 16);
  const int64_t T0 = (int64_t)wk.z * 8 + (L::FULL ? 0 : 4 * wk.w);
  const int64_t nks = (int64_t)(i + 1 - bf) * (TB / 16);
  const int64_t k1 = ph ? nks - 1 : 0;  // first k-step
  constexpr int64_t dir = ph ? -1 : 1;   // direction
  const FragSrc A{it.wa_hi + it.wa_off[i] + k1 * 8 * FRAG, it.wa_lo + it.wa_off[i] + k1 * 8 * FRAG,
                  FRAG, dir * 8 * FRAG};
  const FragSrc B{it.hs_hi + (T0 * it.tks + ks0 + k1) * FRAG,
                  it.hs_lo + (T0 * it.tks + ks0 + k1) * FRAG, it.tks * FRAG, dir * FRAG};
  f16v acc[4][L::WB];
  gemm3_v<3, V>(A, B, nks, tid, acc);
  // element (template b, row p) of F(w0^T): tile b/32, kstep p/16, lane b%32 + 32((p%16)/8),
  // pos p%8.  With two waves per SIMD the thread index is read again, so that no address
  // is held across the product.
  const int tid2 = L::WPS > 1 ? opaque_tid() : tid, lane2 = tid2 & 63, w2 = tid2 >> 6;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t rt_row = (int64_t)i * TB + 32 * (L::ta(w2) + a);
#pragma unroll
    for (int b = 0; b < L::WB; ++b) {
      const int64_t T = T0 + L::tb(w2) + b;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t base = rt_row + 8 * g;
        const int64_t ks = base >> 4;
        const int lp = (lane2 & 31) + 32 * (g & 1);
        const int64_t dst = ((T * it.tks + ks) * 64 + lp) * 8 + 4 * (lane2 >> 5);
        uint16_t h4[4], l4[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) split2f(acc[a][b][4 * g + v], h4[v], l4[v]);
        uint2 vh, vl;
        vh.x = h4[0] | ((uint32_t)h4[1] << 16); vh.y = h4[2] | ((uint32_t)h4[3] << 16);
        vl.x = l4[0] | ((uint32_t)l4[1] << 16); vl.y = l4[2] | ((uint32_t)l4[3] << 16);
        *reinterpret_cast<uint2 *>(it.w0_hi + dst) = vh;
        *reinterpret_cast<uint2 *>(it.w0_lo + dst) = vl;
      }
    }
  }
}

template <int V>
__global__ __launch_bounds__(64 * PL<V>::NW, PL<V>::OCC) void k_trmm_fwd(
    const MixItem *__restrict__ items, const int4 *__restrict__ work) {
  const int4 wk = work[blockIdx.x];
  if (wk.y < 0 || (PL<V>::FULL && wk.w)) return;
  const int np = pair_blocks(items[wk.x], wk.y);
  fwd_block<V, 0>(items, work);
  if (np == 2) fwd_block<V, 1>(items, work);
}

// y0^T = w0^T W over column block j (K = rows [j TB, (last + 1) TB)): A = F(w0^T)
// (256 templates of the group), B = F(W^T) sample tiles of block j (half `sub` for the
// half-group variant).  The first block of the pair (the longer K) walks K downwards from
// the end of the segment, its partner upwards.
template <int V, int ph>
__device__ __forceinline__ void bwd_block(const MixItem *items, const int4 *work) {
  using L = PL<V>;
  const int4 wk = work[blockIdx.x];
  const MixItem &it = items[wk.x];
  const int tid = opaque_tid(), lane = tid & 63, w = tid >> 6;
  const int last = it.blk_last[wk.y];
  const int j = ph ? it.blk_first[wk.y] + last - wk.y : wk.y;
  const int64_t T0 = (int64_t)wk.z * 8;
  const int st0 = L::FULL ? 0 : 4 * wk.w;
  const int64_t nks = (int64_t)(last + 1 - j) * (TB / 16);
  const int64_t ks0 = (int64_t)j * (TB / 16);
  const int64_t k1 = ph ? 0 : nks - 1;  // first k-step
  constexpr int64_t dir = ph ? 1 : -1;   // direction
  const FragSrc A{it.w0_hi + (T0 * it.tks + ks0 + k1) * FRAG,
                  it.w0_lo + (T0 * it.tks + ks0 + k1) * FRAG, it.tks * FRAG, dir * FRAG};
  const FragSrc B{it.wb_hi + it.wb_off[j] + (int64_t)st0 * FRAG + k1 * 8 * FRAG,
                  it.wb_lo + it.wb_off[j] + (int64_t)st0 * FRAG + k1 * 8 * FRAG, FRAG,
                  dir * 8 * FRAG};
  f16v acc[4][L::WB];
  gemm3_v<3, V>(A, B, nks, tid, acc);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t trow0 = 32 * (T0 + L::ta(w) + a);
#pragma unroll
    for (int b = 0; b < L::WB; ++b) {
      const int64_t col = (int64_t)j * TB + 32 * (st0 + L::tb(w) + b) + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t trow = trow0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        it.y0[trow * it.n_pad + col] = acc[a][b][r];
      }
    }
  }
}

template <int V>
__global__ __launch_bounds__(64 * PL<V>::NW, PL<V>::OCC) void k_trmm_bwd(
    const MixItem *__restrict__ items, const int4 *__restrict__ work) {
  const int4 wk = work[blockIdx.x];
  if (wk.y < 0 || (PL<V>::FULL && wk.w)) return;
  const int np = pair_blocks(items[wk.x], wk.y);
  bwd_block<V, 0>(items, work);
  if (np == 2) bwd_block<V, 1>(items, work);
}

// Correction c_b = ||W e_b||^2: the forward product with the split residual (in the
// template buffers) as B; the epilogue writes, per template, the sum of squares over the
// 256 rows of block i to corr_part[i][b] (fixed order, no atomics).  CORR_PROD selects
// 3 (hi*hi + hi*lo + lo*hi) or 1 (hi*hi) products.  Pairs as in the forward product.
constexpr int CORR_PROD = 3;
template <int V, int ph>
__device__ __forceinline__ void corr_block(const MixItem *items, const int4 *work,
                                           double (*red)[256]) {
  using L = PL<V>;
  const int4 wk = work[blockIdx.x];
  const MixItem &it = items[wk.x];
  const int tid = opaque_tid(), lane0 = tid & 63, w0 = tid >> 6;
  const int bf = it.blk_first[wk.y];
  const int i = ph ? bf + it.blk_last[wk.y] - wk.y : wk.y;
  const int64_t ks0 = (int64_t)bf * (TB / 16);
  const int64_t T0 = (int64_t)wk.z * 8 + (L::FULL ? 0 : 4 * wk.w);
  const int64_t nks = (int64_t)(i + 1 - bf) * (TB / 16);
  const int64_t k1 = ph ? nks - 1 : 0;
  constexpr int64_t dir = ph ? -1 : 1;
  const FragSrc A{it.wa_hi + it.wa_off[i] + k1 * 8 * FRAG, it.wa_lo + it.wa_off[i] + k1 * 8 * FRAG,
                  FRAG, dir * 8 * FRAG};
  const FragSrc B{it.es_hi + (T0 * it.tks + ks0 + k1) * FRAG,
                  it.es_lo + (T0 * it.tks + ks0 + k1) * FRAG, it.tks * FRAG, dir * FRAG};
  f16v acc[4][L::WB];
  gemm3_v<CORR_PROD, V>(A, B, nks, tid, acc);
  // per column: sum of squares over the wave's 128 rows; the two row halves of the
  // workgroup meet in LDS.  With two waves per SIMD the thread index is read again, as in
  // the forward product.
  const int tid2 = L::WPS > 1 ? opaque_tid() : tid;
  const int lane = L::WPS > 1 ? tid2 & 63 : lane0, w = L::WPS > 1 ? tid2 >> 6 : w0;
#pragma unroll
  for (int b = 0; b < L::WB; ++b) {
    double ss = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) ss += (double)acc[a][b][r] * (double)acc[a][b][r];
    ss += __shfl_xor(ss, 32);  // lanes l and l+32 hold other rows of the same column
    const int col = 32 * (L::tb(w) + b) + (lane & 31);
    if (lane < 32) red[L::ta(w) >> 2][col] = ss;
  }
  __syncthreads();
  const int ncol = L::FULL ? 256 : 128;
  for (int col = tid2; col < ncol; col += 64 * L::NW)
    it.corr_part[(int64_t)i * it.Bp + T0 * 32 + col] = red[0][col] + red[1][col];
}

// LDS for the column sums: the LDS variant uses its operand ring, idle by then (a static
// array would not fit beside its stages)
template <int V>
__device__ __forceinline__ double (*corr_red())[256] {
  if constexpr (PL<V>::LDS_STAGES > 0) {
    extern __shared__ char gp_smem[];
    return (double (*)[256])gp_smem;
  } else {
    __shared__ double red[2][256];
    return red;
  }
}

template <int V>
__global__ __launch_bounds__(64 * PL<V>::NW, PL<V>::OCC) void k_corr(
    const MixItem *__restrict__ items, const int4 *__restrict__ work) {
  double (*red)[256] = corr_red<V>();
  const int4 wk = work[blockIdx.x];
  if (wk.y < 0 || (PL<V>::FULL && wk.w)) return;
  const int np = pair_blocks(items[wk.x], wk.y);
  corr_block<V, 0>(items, work, red);
  if (np == 2) {
    __syncthreads();  // the first block's sums have been read
    corr_block<V, 1>(items, work, red);
  }
}

// out[b] = -1/2 (qpart[b] + sum_i corr_part[i][b]) + cterm; entries (item, b).  With
// hh_out, the refinement left the refined h^T C^-1 h there and the correction is added.
__global__ void k_finish(const MixItem *__restrict__ items, const int2 *__restrict__ work,
                         int64_t n_work) {
  const int64_t wi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (wi >= n_work) return;
  const int2 wk = work[wi];
  const MixItem &it = items[wk.x];
  const int64_t b = wk.y;
  double c = 0.0;
  for (int i = 0; i < it.nblk; ++i) c += it.corr_part[(int64_t)i * it.Bp + b];
  it.out[b] = -0.5 * (it.qpart[b] + c) + it.cterm;
  if (it.hh_out) it.hh_out[b] += c;  // refined h^T C^-1 h plus the correction
}

#define TDA_LAUNCH_VARIANT(K)                                                                 \
  if (n_work <= 0) return hipSuccess;                                                        \
  switch (variant) {                                                                         \
    case 2:                                                                                  \
      hipLaunchKernelGGL(K<2>, dim3((unsigned)n_work), dim3(256), 0, s, items, work);         \
      break;                                                                                 \
    case 4:                                                                                  \
      hipLaunchKernelGGL(K<4>, dim3((unsigned)n_work), dim3(256), 0, s, items, work);         \
      break;                                                                                 \
    case 5:                                                                                  \
      hipLaunchKernelGGL(K<5>, dim3((unsigned)n_work), dim3(512), PL<5>::lds_bytes(), s,     \
                         items, work);                                                       \
      break;                                                                                 \
    default:                                                                                 \
      hipLaunchKernelGGL(K<1>, dim3((unsigned)n_work), dim3(256), 0, s, items, work);         \
  }                                                                                          \
  return hipGetLastError();

hipError_t launch_trmm_fwd(const MixItem *items, const int4 *work, int64_t n_work, int variant,
                           hipStream_t s) {
  TDA_LAUNCH_VARIANT(k_trmm_fwd)
}

hipError_t launch_trmm_bwd(const MixItem *items, const int4 *work, int64_t n_work, int variant,
                           hipStream_t s) {
  TDA_LAUNCH_VARIANT(k_trmm_bwd)
}

hipError_t launch_corr(const MixItem *items, const int4 *work, int64_t n_work, int variant,
                       hipStream_t s) {
  TDA_LAUNCH_VARIANT(k_corr)
}

hipError_t launch_finish(const MixItem *items, const int2 *work, int64_t n_work, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finish, dim3((unsigned)((n_work + 255) / 256)), dim3(256), 0, s, items,
                     work, n_work);
  return hipGetLastError();
}


// ---------------------------------------------------------------- FP64 refinement
// Per template pair (a, b) and segment: x = y0 scattered to the segment's sample
// positions (0 at excluded samples and beyond the segment), z = x_a + i x_b, and
//   C x = first `length` entries of IDFT_m(lambda . DFT_m(z))   (real part: a, imag: b)
// because C is the leading block of the circulant of length m >= 2 length whose first
// column embeds the ACF (eq:toeplitz_fft; lambda is real and even, so the two real
// sequences separate in the real and imaginary parts).  With e = h - C y0 (FP64):
//   s_hat = 2 h^T y0 - y0^T C y0 <= h^T C^-1 h, error (y* - y0)^T C (y* - y0) = e^T C^-1 e,
// the correction kernel adds ||W e||^2, and the remaining error is third order.
//   qpart = q_dd - 2 y_d^T h + s_hat        (FP64); e is written for the correction.
// Length-m DFTs are four-step (m = n1 n2): n1-point DFTs down the columns of x seen as
// n1 x n2 row-major, twiddle w_m^{j2 k1}, n2-point DFTs along the rows; the inverse runs
// the same steps backwards (conjugation trick).  Each n-point DFT (n <= 512) is itself
// two register DFTs of P1 <= 16 and P2 <= 32 points with one LDS exchange; the length-m
// intermediate lives in the workgroup's global scratch.

constexpr int RF_THREADS = 128;
constexpr int RF_LDS = 2048;  // complex doubles in the LDS work buffer

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

__host__ __device__ constexpr int brev_c(int x, int L) {
  int r = 0;
  for (int i = 0; i < L; ++i) r |= ((x >> i) & 1) << (L - 1 - i);
  return r;
}

// Forward DFT of 2^L points held in registers, decimation in frequency: natural order
// in, bit-reversed order out (X[k] ends in v[brev(k)]; the callers index accordingly).
// twP[k] = exp(-2 pi i k / P) for the enclosing length P = 2^LP (LP >= L).
template <int L, int LP>
__device__ __forceinline__ void dft_reg(double2 (&v)[1 << L], const double2 *twP) {
  constexpr int N = 1 << L;
#pragma unroll
  for (int s = L; s >= 1; --s) {
    const int half = 1 << (s - 1), span = 1 << s;
#pragma unroll
    for (int g = 0; g < N; g += span)
#pragma unroll
      for (int o = 0; o < half; ++o) {
        const double2 a = v[g + o], b = v[g + o + half];
        v[g + o] = cadd(a, b);
        const double2 d = csub(a, b);
        v[g + o + half] = o ? cmul(d, twP[o << (LP - s)]) : d;  // exp(-2 pi i o / span)
      }
  }
}

// In-place forward DFTs of `cols` sequences of length P = 2^(L1 + L2) at X[c P + j]
// (natural order in and out): j = P2 j1 + j2, k = k1 + P1 k2.  Needs cols P2 <= threads
// and cols P1 <= threads.
template <int L1, int L2>
__device__ __forceinline__ void dft_cols(double2 *X, int cols, const double2 *twP) {
  constexpr int P1 = 1 << L1, P2 = 1 << L2, P = P1 * P2, LP = L1 + L2;
  const int t = threadIdx.x;
  // step 1: item (c, j2): DFT over j1, twiddle w_P^{j2 k1}, to X[c P + k1 P2 + j2]
  {
    const bool act = t < cols * P2;
    const int c = t >> L2, j2 = t & (P2 - 1);
    double2 v[P1];
    if (act) {
#pragma unroll
      for (int j1 = 0; j1 < P1; ++j1) v[j1] = X[c * P + P2 * j1 + j2];
      dft_reg<L1, LP>(v, twP);
#pragma unroll
      for (int k1 = 1; k1 < P1; ++k1)
        v[brev_c(k1, L1)] = cmul(v[brev_c(k1, L1)], twP[(j2 * k1) & (P - 1)]);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int k1 = 0; k1 < P1; ++k1) X[c * P + k1 * P2 + j2] = v[brev_c(k1, L1)];
    }
    __syncthreads();
  }
  // step 2: item (c, k1): DFT over j2, to X[c P + k1 + P1 k2]
  {
    const bool act = t < cols * P1;
    const int c = t >> L1, k1 = t & (P1 - 1);
    double2 u[P2];
    if (act) {
#pragma unroll
      for (int j2 = 0; j2 < P2; ++j2) u[j2] = X[c * P + k1 * P2 + j2];
      dft_reg<L2, LP>(u, twP);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int k2 = 0; k2 < P2; ++k2) X[c * P + k1 + P1 * k2] = u[brev_c(k2, L2)];
    }
    __syncthreads();
  }
}

__device__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

struct PairAcc {
  double hy_a, hy_b, ydh_a, ydh_b, yc_a, yc_b, bad_a, bad_b;
};

// log2 of the register factors of an n-point DFT: P1 = 2^min(L, 4), P2 = 2^(L - that)
template <int L> struct Split { static constexpr int A = L < 4 ? L : 4; static constexpr int B = L - A; };

template <int LM>
__device__ void refine_segment(const RefItem &it, const SegDev &sd, int64_t ba, int64_t bb,
                               bool two, double2 *X, double2 *tw1, double2 *tw2, double2 *S,
                               PairAcc &acc) {
  constexpr int L1 = (LM + 1) / 2, L2 = LM / 2;
  constexpr int n1 = 1 << L1, n2 = 1 << L2;
  constexpr int64_t m = (int64_t)1 << LM;
  constexpr int A1 = Split<L1>::A, B1 = Split<L1>::B, A2 = Split<L2>::A, B2 = Split<L2>::B;
  // columns per LDS batch (each register step needs cols * P <= threads)
  constexpr int cmax1 = RF_THREADS / ((1 << A1) > (1 << B1) ? (1 << A1) : (1 << B1));
  constexpr int cb1 = (cmax1 < RF_LDS / n1 ? cmax1 : RF_LDS / n1) < n2 ? (cmax1 < RF_LDS / n1 ? cmax1 : RF_LDS / n1) : n2;
  constexpr int cmax2 = RF_THREADS / ((1 << A2) > (1 << B2) ? (1 << A2) : (1 << B2));
  constexpr int cb2 = (cmax2 < RF_LDS / n2 ? cmax2 : RF_LDS / n2) < n1 ? (cmax2 < RF_LDS / n2 ? cmax2 : RF_LDS / n2) : n1;
  const float *ya = it.y0 + ba * it.n_pad;
  const float *yb = it.y0 + (two ? bb : ba) * it.n_pad;
  const double *ha = template_row(it, ba);
  const double *hb = template_row(it, two ? bb : ba);
  const EsOut ea(it.es_hi, it.es_lo, it.tks, ba);
  const EsOut eb(it.es_hi, it.es_lo, it.tks, two ? bb : ba);
  for (int k = threadIdx.x; k < n1; k += blockDim.x) {
    const int64_t r = (int64_t)k * (m / n1);
    tw1[k] = make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]);
  }
  for (int k = threadIdx.x; k < n2; k += blockDim.x) {
    const int64_t r = (int64_t)k * (m / n2);
    tw2[k] = make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]);
  }
  // padded rows of the segment carry e = 0
  for (int64_t p = sd.row0 + sd.nkeep + threadIdx.x; p < sd.row0 + sd.npad; p += blockDim.x) {
    ea.put((int32_t)p, 0.0);
    if (two) eb.put((int32_t)p, 0.0);
  }
  __syncthreads();
  // pass 1: column DFTs (length n1) of x[n2 j1 + j2], twiddle w_m^{j2 k1}, to S[k1 n2 + j2]
  for (int j2b = 0; j2b < n2; j2b += cb1) {
    for (int u = threadIdx.x; u < cb1 * n1; u += blockDim.x) {
      const int c = u % cb1, j1 = u / cb1;
      const int64_t jpos = (int64_t)n2 * j1 + j2b + c;
      double xa = 0.0, xb = 0.0;
      if (jpos < sd.length) {
        const int32_t p = it.pos2row[sd.offset + jpos];
        if (p >= 0) {
          xa = (double)ya[p];
          if (!isfinite(xa)) acc.bad_a = 1.0, xa = 0.0;
          if (two) {
            xb = (double)yb[p];
            if (!isfinite(xb)) acc.bad_b = 1.0, xb = 0.0;
          }
        }
      }
      X[c * n1 + j1] = make_double2(xa, xb);
    }
    __syncthreads();
    dft_cols<A1, B1>(X, cb1, tw1);
    for (int u = threadIdx.x; u < cb1 * n1; u += blockDim.x) {
      const int c = u % cb1, k1 = u / cb1;
      const int64_t j2 = j2b + c;
      const int64_t r = (j2 * (int64_t)k1) & (m - 1);
      S[(int64_t)k1 * n2 + j2] = cmul(X[c * n1 + k1], make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]));
    }
    __syncthreads();
  }
  // pass 2: row DFTs (length n2), times lambda, inverse row DFTs (conjugated), twiddle
  for (int k1b = 0; k1b < n1; k1b += cb2) {
    for (int u = threadIdx.x; u < cb2 * n2; u += blockDim.x) {
      const int c = u / n2, j2 = u % n2;
      X[c * n2 + j2] = S[(int64_t)(k1b + c) * n2 + j2];
    }
    __syncthreads();
    dft_cols<A2, B2>(X, cb2, tw2);
    for (int u = threadIdx.x; u < cb2 * n2; u += blockDim.x) {
      const int c = u / n2, k2 = u % n2;
      const double lam = sd.lam[(int64_t)(k1b + c) + (int64_t)n1 * k2];
      const double2 v = X[c * n2 + k2];
      X[c * n2 + k2] = make_double2(lam * v.x, -lam * v.y);  // conj(lambda X)
    }
    __syncthreads();
    dft_cols<A2, B2>(X, cb2, tw2);
    for (int u = threadIdx.x; u < cb2 * n2; u += blockDim.x) {
      const int c = u / n2, j2 = u % n2;
      const int64_t k1 = k1b + c;
      const int64_t r = (k1 * (int64_t)j2) & (m - 1);
      // inverse row result = conj(X); times w_m^{-j2 k1}; stored conjugated for pass 3
      S[k1 * n2 + j2] = cmul(X[c * n2 + j2], make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]));
    }
    __syncthreads();
  }
  // pass 3: inverse column DFTs (length n1) -> (C z) at positions n2 j1 + j2; residual and dots
  const double inv_m = 1.0 / (double)m;
  for (int j2b = 0; j2b < n2; j2b += cb1) {
    for (int u = threadIdx.x; u < cb1 * n1; u += blockDim.x) {
      const int c = u % cb1, k1 = u / cb1;
      X[c * n1 + k1] = S[(int64_t)k1 * n2 + j2b + c];
    }
    __syncthreads();
    dft_cols<A1, B1>(X, cb1, tw1);
    for (int u = threadIdx.x; u < cb1 * n1; u += blockDim.x) {
      const int c = u % cb1, j1 = u / cb1;
      const int64_t jpos = (int64_t)n2 * j1 + j2b + c;
      if (jpos >= sd.length) continue;
      const int64_t jg = sd.offset + jpos;
      const int32_t p = it.pos2row[jg];
      if (p < 0) continue;
      const double2 v = X[c * n1 + j1];
      const double cza = v.x * inv_m, czb = -v.y * inv_m;
      const double yd = it.yd_pos[jg];
      const double xa = (double)ya[p];
      const double hva = ha[jg];
      ea.put(p, hva - cza);
      acc.hy_a += hva * xa;
      acc.ydh_a += hva * yd;
      acc.yc_a += xa * cza;
      if (two) {
        const double xb = (double)yb[p];
        const double hvb = hb[jg];
        eb.put(p, hvb - czb);
        acc.hy_b += hvb * xb;
        acc.ydh_b += hvb * yd;
        acc.yc_b += xb * czb;
      }
    }
    __syncthreads();
  }
}

// Work entry: (item, template a, template b or -1, 0).  Persistent grid; each workgroup
// owns m complex doubles of scratch.  Used for launches with a circulant longer than the
// in-LDS refinement takes (m > 65536).
// LMAX bounds log2 m of the segments the instantiation handles (register DFTs of up to
// 2^(LMAX/2 - 4) points).
template <int LMAX>
__global__ __launch_bounds__(RF_THREADS) void k_refine(const RefItem *__restrict__ items,
                                                       const int4 *__restrict__ work,
                                                       int64_t n_work,
                                                       double2 *__restrict__ scratch_all,
                                                       int64_t scratch_per_wg) {
  __shared__ double2 X[RF_LDS];
  __shared__ double2 tw1[512], tw2[512];
  __shared__ double red[RF_THREADS];
  double2 *S = scratch_all + (int64_t)blockIdx.x * scratch_per_wg;
  for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
    const int4 wk = work[wi];
    const RefItem &it = items[wk.x];
    const int64_t ba = wk.y, bb = wk.z;
    const bool two = bb >= 0;
    PairAcc acc{0, 0, 0, 0, 0, 0, 0, 0};
    for (int sg = 0; sg < it.n_segs; ++sg) {
      const SegDev sd = it.segs[sg];
      switch (sd.log2m) {
#define TDA_SEG(LM)                                                             \
  case LM:                                                                      \
    if constexpr (LM <= LMAX) refine_segment<LM>(it, sd, ba, bb, two, X, tw1, tw2, S, acc); \
    else acc.bad_a = acc.bad_b = 1.0;                                           \
    break;
        TDA_SEG(1) TDA_SEG(2) TDA_SEG(3) TDA_SEG(4) TDA_SEG(5) TDA_SEG(6) TDA_SEG(7)
        TDA_SEG(8) TDA_SEG(9) TDA_SEG(10) TDA_SEG(11) TDA_SEG(12) TDA_SEG(13) TDA_SEG(14)
        TDA_SEG(15) TDA_SEG(16) TDA_SEG(17) TDA_SEG(18)
#undef TDA_SEG
        default: acc.bad_a = acc.bad_b = 1.0;
      }
    }
    const double s_hya = block_sum(acc.hy_a, red), s_ydha = block_sum(acc.ydh_a, red);
    const double s_yca = block_sum(acc.yc_a, red);
    const double s_hyb = block_sum(acc.hy_b, red), s_ydhb = block_sum(acc.ydh_b, red);
    const double s_ycb = block_sum(acc.yc_b, red);
    const double s_bada = block_sum(acc.bad_a, red), s_badb = block_sum(acc.bad_b, red);
    if (threadIdx.x == 0) {
      const double nan = __builtin_nan("");
      it.qpart[ba] = s_bada > 0 ? nan : it.qdd[0] - 2.0 * s_ydha + 2.0 * s_hya - s_yca;
      if (two) it.qpart[bb] = s_badb > 0 ? nan : it.qdd[0] - 2.0 * s_ydhb + 2.0 * s_hyb - s_ycb;
      if (it.dh_out) {
        // a NaN q_dd marks data that the handle can no longer whiten: <d,h> is NaN too
        const bool dbad = isnan(it.qdd[0]);
        it.dh_out[ba] = s_bada > 0 || dbad ? nan : s_ydha;
        if (two) it.dh_out[bb] = s_badb > 0 || dbad ? nan : s_ydhb;
      }
      if (it.hh_out) {
        it.hh_out[ba] = s_bada > 0 ? nan : 2.0 * s_hya - s_yca;
        if (two) it.hh_out[bb] = s_badb > 0 ? nan : 2.0 * s_hyb - s_ycb;
      }
    }
  }
}

hipError_t launch_refine(const RefItem *items, const int4 *work, int64_t n_work, double *scratch,
                         int64_t scratch_per_wg, int32_t n_wg, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine<18>, dim3((unsigned)n_wg), dim3(RF_THREADS), 0, s, items, work,
                     n_work, (double2 *)scratch, scratch_per_wg / 2);
  return hipGetLastError();
}

// ---------------------------------------------------------------- FP64 refinement in LDS
// Same quantities as k_refine (C y0 by circulant embedding, eq:toeplitz_fft), organised so
// that one template's transforms fit in one workgroup's LDS.  With m = 4h the circulant
// length, n' = m/2 >= length, w_m = exp(-2 pi i / m) and x = y0 at the segment's sample
// positions (0 at excluded samples and beyond the segment):
//   (C x)_j = (1/m) [ tE_j + tO_j ],   j < length,
//   tE = unnormalised inverse n'-point DFT of (lambda_{2k} X_{2k})     (circulant part)
//   tO_j = sum_{k < n'} lambda_{2k+1} X_{2k+1} w_m^{-j(2k+1)}          (skew-circulant part)
// where X_r = sum_j x_j w_m^{j r}.  Each part is one forward and one inverse h-point
// complex DFT of the real data packed as x_{2p} + i x_{2p+1} (pre-multiplied by w_m^{2p}
// for the odd part); the pointwise stage between them pairs index k with h-k (even part)
// or h-1-k (odd part), whose values are conjugate-symmetric.  Inverse DFTs are forward
// DFTs of the conjugate.  The h-point DFT is a sequence of in-place Stockham passes over
// an LDS array padded by one element per 16 (bank spread for the strided writes).
constexpr int RL_THREADS = 512;
constexpr int RL_XN = (1 << RL_LHMAX) + ((1 << RL_LHMAX) >> 4);
constexpr int RL_RED = 4 * (RL_THREADS / 64);  // per-wave partial sums, up to 4 values
constexpr size_t RL_LDS_BYTES = (size_t)RL_XN * sizeof(double2) + RL_RED * sizeof(double);

// Sums of K values over the workgroup, valid on thread 0 only: a butterfly within each
// wave, then thread 0 adds the waves' partial sums in wave order (so the result does not
// depend on timing).  Ends with a barrier, so `red` may be reused at once.
template <int K>
__device__ __forceinline__ void block_sum0(double (&v)[K], double *red) {
  static_assert(K * (RL_THREADS / 64) <= RL_RED, "partial sums fit");
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] += __shfl_xor(v[i], o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < K; ++i) red[w * K + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      double a = red[i];
      for (int u = 1; u < (int)(blockDim.x >> 6); ++u) a += red[u * K + i];
      v[i] = a;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 scal(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 mul_i(double2 a) { return make_double2(-a.y, a.x); }

// cos(pi t / 16) for 0 <= t <= 16 (correctly rounded doubles).
__device__ __forceinline__ constexpr double cos_pi16(int t) {
  const int u = t <= 8 ? t : 16 - t;
  const double c = u == 0 ? 1.0 : u == 1 ? 0x1.f6297cff75cb0p-1 : u == 2 ? 0x1.d906bcf328d46p-1
                 : u == 3 ? 0x1.a9b66290ea1a3p-1 : u == 4 ? 0x1.6a09e667f3bcdp-1
                 : u == 5 ? 0x1.1c73b39ae68c8p-1 : u == 6 ? 0x1.87de2a6aea963p-2
                 : u == 7 ? 0x1.8f8b83c69a60bp-3 : 0.0;
  return t <= 8 ? c : -c;
}

// Forward DFT of 2^L <= 32 points in registers, decimation in frequency, natural order in,
// bit-reversed order out; the twiddles w_32^t are constants, so they cost no registers and
// the trivial ones (1, -i) no multiplications.
template <int L>
__device__ __forceinline__ void dft_small(double2 (&v)[1 << L]) {
  static_assert(L <= 5, "at most 32 points");
  constexpr int N = 1 << L;
#pragma unroll
  for (int s = L; s >= 1; --s) {
    const int half = 1 << (s - 1), span = 1 << s;
#pragma unroll
    for (int g = 0; g < N; g += span)
#pragma unroll
      for (int o = 0; o < half; ++o) {
        const double2 a = v[g + o], b = v[g + o + half];
        v[g + o] = cadd(a, b);
        const double2 d = csub(a, b);
        const int t = (32 / span) * o;  // w_span^o = w_32^t = cos(pi t/16) - i sin(pi t/16)
        if (t == 0) {
          v[g + o + half] = d;
        } else if (t == 8) {
          v[g + o + half] = make_double2(d.y, -d.x);
        } else {
          const double c = cos_pi16(t), sn = cos_pi16(t < 8 ? 8 - t : t - 8);
          v[g + o + half] = make_double2(d.x * c + d.y * sn, d.y * c - d.x * sn);
        }
      }
  }
}

// Pass P of the h = 2^LH point forward DFT: radix R = 2^L over sub-transforms of length
// Ns = 2^LNS.  Sub-transform j < h/R loads X[j + q h/R], twiddles by w_{Ns R}^{q (j mod Ns)},
// transforms, and stores to X[(j div Ns) Ns R + j mod Ns + q Ns] (natural order at the end).
// Thread t takes j = t + RL_THREADS g, g < G; every element is read into registers before
// any is written back, so the pass works in place.
template <int LH, int P>
__device__ __forceinline__ void rl_pass(double2 *X, const gmem<const dv2> *__restrict__ ptw) {
  constexpr int L = rl_L(LH, P), LNS = rl_lns(LH, P), OFF = rl_off(LH, P);
  constexpr int R = 1 << L, NS = 1 << LNS, NT = 1 << (LH - L);
  constexpr int G = NT > RL_THREADS ? NT / RL_THREADS : 1;
  constexpr int NTA = NT > RL_THREADS ? RL_THREADS : NT;
  const int t = threadIdx.x;
  const bool act = t < NTA;
  double2 a[G][R];
  if (act) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = t + RL_THREADS * g, k = j & (NS - 1);
      // strides that are multiples of 16 keep the padded addresses at constant offsets
      if constexpr (NT % 16 == 0) {
        const double2 *x0 = X + lpad(j);
#pragma unroll
        for (int q = 0; q < R; ++q) a[g][q] = x0[q * (NT + NT / 16)];
      } else {
#pragma unroll
        for (int q = 0; q < R; ++q) a[g][q] = X[lpad(j + q * NT)];
      }
      if constexpr (LNS > 0) {
        // a few twiddles at a time, so they do not all hold registers at once
        const gmem<const dv2> *tk = ptw + OFF + k * (R - 1);
#pragma unroll
        for (int q = 1; q < R; ++q) {
          a[g][q] = cmul(a[g][q], from_dv2(tk[q - 1]));
          if (q % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
      }
      dft_small<L>(a[g]);
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = t + RL_THREADS * g, k = j & (NS - 1);
      const int base = ((j >> LNS) << (LNS + L)) + k;
      if constexpr (NS % 16 == 0) {
        double2 *x0 = X + lpad(base);
#pragma unroll
        for (int q = 0; q < R; ++q) x0[q * (NS + NS / 16)] = a[g][brev_c(q, L)];
      } else if constexpr (NS == 1 && R % 16 == 0) {
        double2 *x0 = X + lpad(base);  // base = j R, a multiple of 16
#pragma unroll
        for (int q = 0; q < R; ++q) x0[q + (q >> 4)] = a[g][brev_c(q, L)];
      } else {
#pragma unroll
        for (int q = 0; q < R; ++q) X[lpad(base + q * NS)] = a[g][brev_c(q, L)];
      }
    }
  }
  __syncthreads();
}

template <int LH>
__device__ __forceinline__ void rl_fft(double2 *X, const gmem<const dv2> *ptw) {
  static_assert(rl_npass(LH) <= 4, "at most four passes");
  rl_pass<LH, 0>(X, ptw);
  if constexpr (rl_npass(LH) > 1) rl_pass<LH, 1>(X, ptw);
  if constexpr (rl_npass(LH) > 2) rl_pass<LH, 2>(X, ptw);
  if constexpr (rl_npass(LH) > 3) rl_pass<LH, 3>(X, ptw);
}

struct RlAcc {
  double hy, ydh, yc, bad;
};

// Multiplier of the circulant product: real eigenvalues (the covariance) or complex
// spectra (the Gohberg-Semencul correlations).
__device__ __forceinline__ double2 mulm(double a, double2 v) { return scal(a, v); }
__device__ __forceinline__ double2 mulm(double2 a, double2 v) { return cmul(a, v); }

// Pointwise stage of the circulant (even-frequency) part for the pair (k, h - k) of the
// packed h-point spectrum: vk = Z_k, vr = Z_{h-k}, la = lambda_{2k}, lb = lambda_{2h-2k},
// cc = w_m^{2k}.  The spectra of the even- and odd-indexed samples are
// E = (vk + conj vr)/2 and O = -i (vk - conj vr)/2; gk, gr are the conjugated inputs of the
// inverse DFT at k and h - k (for k = 0 or h/2 the pair is one index and gr is unused).
template <class Mul>
__device__ __forceinline__ void rl_even_pair(double2 vk, double2 vr, Mul la, Mul lb,
                                             double2 cc, double2 &gk, double2 &gr) {
  const double2 E = make_double2(0.5 * (vk.x + vr.x), 0.5 * (vk.y - vr.y));
  const double2 O = make_double2(0.5 * (vk.y + vr.y), -0.5 * (vk.x - vr.x));
  const double2 cO = cmul(cc, O);
  const double2 yk = mulm(la, cadd(E, cO));
  const double2 yr = mulm(lb, conj2(csub(E, cO)));
  const double2 ep = cadd(yk, conj2(yr)), op = csub(yk, conj2(yr));
  gk = conj2(cadd(ep, mul_i(cmul(conj2(cc), op))));
  gr = conj2(cadd(conj2(ep), mul_i(cmul(cc, conj2(op)))));
}

// Pointwise stage of the skew-circulant (odd-frequency) part for the pair (k, h - 1 - k):
// vk = Z_k, vr = Z_{h-1-k}, la = lambda_{2k+1}, lb = lambda_{2k+2h+1}, dd = w_m^{2k+1},
// cc = w_m^{2k}, om = w_m; gk, gr as for the even part.
template <class Mul>
__device__ __forceinline__ void rl_odd_pair(double2 vk, double2 vr, Mul la, Mul lb, double2 dd,
                                            double2 cc, double2 om, double2 &gk, double2 &gr) {
  const double2 A = make_double2(0.5 * (vk.x + vr.x), 0.5 * (vk.y - vr.y));
  const double2 B = make_double2(0.5 * (vk.y + vr.y), -0.5 * (vk.x - vr.x));
  const double2 dB = cmul(dd, B);
  const double2 yk = mulm(la, cadd(A, dB));   // X_{2k+1}
  const double2 ykh = mulm(lb, csub(A, dB));  // X_{2k+2h+1}
  const double2 P = cadd(yk, ykh);
  const double2 Q = cmul(conj2(cc), csub(yk, ykh));
  gk = conj2(cadd(P, mul_i(cmul(conj2(om), Q))));
  gr = conj2(cadd(conj2(P), mul_i(cmul(om, conj2(Q)))));
}

// Element-wise phases: a thread handles positions p = t + RL_THREADS i (samples 2p and
// 2p + 1) or frequency pairs k = t + RL_THREADS i.  A phase issues the device-memory
// accesses of a whole batch of positions before it uses any of them, so it waits for
// memory once per batch: the phases that read y0 (or nothing) and the pointwise ones take
// up to RL_CHL positions at once (all of a thread's at h = 8192), the final phase, which
// reads four arrays, RL_CHF.  (Stores to e would otherwise keep later loads from being
// hoisted above them.)  Segments without excluded samples compute rows instead of loading
// them, and read a sample pair's y0 values as one vector (the pair's first row is even
// there).  The residual e goes out split, in the products' fragment layout (EsOut).
constexpr int RL_CH = 4;    // batch of the split transforms' phases
constexpr int RL_CHL = 16;  // batch of the in-LDS phases that read y0 only, and pointwise ones
constexpr int RL_CHF = 8;   // batch of the final in-LDS phase

typedef float fv2 __attribute__((ext_vector_type(2)));

template <int LH>
__device__ __noinline__ void rl_segment(const RefItem &it, const SegDev &sd, int64_t b, double2 *X,
                           RlAcc &acc) {
  constexpr int h = 1 << LH;
  constexpr int NI = h >= RL_THREADS ? h / RL_THREADS : 1;         // position iterations
  constexpr int NKE = (h / 2 + RL_THREADS) / RL_THREADS;           // k = 0 .. h/2
  constexpr int NKO = h / 2 >= RL_THREADS ? h / 2 / RL_THREADS : 1; // k = 0 .. h/2 - 1
  constexpr int CL = NI < RL_CHL ? NI : RL_CHL;
  constexpr int CF = NI < RL_CHF ? NI : RL_CHF;
  constexpr int CKE = NKE < RL_CHL ? NKE : RL_CHL;
  constexpr int CKO = NKO < RL_CHL ? NKO : RL_CHL;
  // the thread index is re-read (opaquely) at each phase, so that per-position rows, masks
  // and addresses are recomputed there rather than held in registers across phases
  int t = opaque_tid();
  const gmem<const float> *__restrict__ y = gpu(it.y0 + b * it.n_pad);
  const gmem<const double> *__restrict__ hrow = gpu(template_row(it, b) + sd.offset);
  const gmem<const double> *__restrict__ ydp = gpu(it.yd_pos + sd.offset);
  const gmem<const int32_t> *__restrict__ p2r = gpu(it.pos2row + sd.offset);
  const EsOut es(it.es_hi, it.es_lo, it.tks, b);
  const gmem<const dv2> *__restrict__ tw = gpu((const dv2 *)sd.tw);  // (cos, sin) of 2 pi r / m
  const gmem<const dv2> *__restrict__ ptw = gpu((const dv2 *)sd.ptw);
  const gmem<const double> *__restrict__ lam = gpu(sd.lam);
  const int len = uni((int)sd.length);
  const bool dense = uni((int)(sd.nkeep == sd.length)) != 0;
  const int32_t row0 = uni((int32_t)sd.row0);
  const double inv_m = 1.0 / (double)(4 * h);
  // sums kept in registers here and added to the caller's at the end (through the reference
  // every update would be a store to memory)
  RlAcc a{0, 0, 0, 0};
  auto wm = [&](int r) {  // w_m^r, 0 <= r < m
    const dv2 v = tw[r];
    return make_double2(v.x, -v.y);
  };
  auto in_pos = [&](int i) { return i < NI && t + RL_THREADS * i < h; };
  // padded rows of samples 2p, 2p + 1 of position i; -1 if excluded or beyond the segment
  auto rows = [&](int i, int32_t (&r)[2]) {
    const int jj = 2 * (t + RL_THREADS * i);
    const bool in = in_pos(i);
#pragma unroll
    for (int u = 0; u < 2; ++u)
      r[u] = !in || jj + u >= len ? -1 : dense ? row0 + jj + u : p2r[jj + u];
  };
  // y0 at rows r (0 where excluded)
  auto load_y = [&](const int32_t (&r)[2]) -> fv2 {
    fv2 v;
    if (dense && r[1] >= 0) {
      v = *(const gmem<const fv2> *)(y + r[0]);
    } else {
      v.x = r[0] >= 0 ? y[r[0]] : 0.f;
      v.y = r[1] >= 0 ? y[r[1]] : 0.f;
    }
    return v;
  };
  auto finite_or_flag = [&](float v) -> double {
    if (!isfinite(v)) {
      a.bad = 1.0;
      return 0.0;
    }
    return (double)v;
  };
  // A thread's sample pairs keep their y0 values and the circulant part t_E / m in
  // registers from the phase that produces them to the final one, so y0 is read from
  // device memory once and t_E never goes there.
  fv2 yk[NI];
  double2 te[NI];

  for (int64_t q = sd.row0 + sd.nkeep + t; q < sd.row0 + sd.npad; q += RL_THREADS)
    es.put((int32_t)q, 0.0);

  // ---- even frequencies: circulant part
  t = opaque_tid();
#pragma unroll
  for (int i0 = 0; i0 < NI; i0 += CL) {
    int32_t r[CL][2];
#pragma unroll
    for (int c = 0; c < CL; ++c) rows(i0 + c, r[c]);
#pragma unroll
    for (int c = 0; c < CL; ++c) yk[i0 + c] = load_y(r[c]);
#pragma unroll
    for (int c = 0; c < CL; ++c) {
      if (!in_pos(i0 + c)) continue;
      X[lpad(t + RL_THREADS * (i0 + c))] =
          make_double2(finite_or_flag(yk[i0 + c].x), finite_or_flag(yk[i0 + c].y));
    }
  }
  __syncthreads();
  rl_fft<LH>(X, ptw);
  t = opaque_tid();
  for (int i0 = 0; i0 < NKE; i0 += CKE) {
    double la[CKE], lb[CKE];
    double2 cc[CKE];
#pragma unroll
    for (int c = 0; c < CKE; ++c) {
      const int k = t + RL_THREADS * (i0 + c);
      if (i0 + c < NKE && k <= h / 2) {
        la[c] = lam[2 * k];
        lb[c] = lam[2 * h - 2 * k];
        cc[c] = wm(2 * k);  // w_{n'}^k
      }
    }
#pragma unroll
    for (int c = 0; c < CKE; ++c) {
      const int k = t + RL_THREADS * (i0 + c);
      if (!(i0 + c < NKE && k <= h / 2)) continue;
      const int kr = (h - k) & (h - 1);
      double2 gk, gr;
      rl_even_pair(X[lpad(k)], X[lpad(kr)], la[c], lb[c], cc[c], gk, gr);
      X[lpad(k)] = gk;
      if (k != 0 && k != h / 2) X[lpad(kr)] = gr;
    }
  }
  __syncthreads();
  rl_fft<LH>(X, ptw);
  // tE_{2p} + i tE_{2p+1} = conj(X[p]), then the odd part's input over it: each thread
  // reads and writes only its own positions here, so no barrier between the two
  t = opaque_tid();
  const double2 om = wm(1);
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    if (!in_pos(i)) continue;
    const int p = t + RL_THREADS * i;
    const double2 v = X[lpad(p)];
    te[i] = make_double2(v.x * inv_m, -v.y * inv_m);
    const double2 z = make_double2(isfinite(yk[i].x) ? (double)yk[i].x : 0.0,
                                   isfinite(yk[i].y) ? (double)yk[i].y : 0.0);
    X[lpad(p)] = cmul(z, wm(2 * p));
  }
  __syncthreads();

  // ---- odd frequencies: skew-circulant part
  rl_fft<LH>(X, ptw);
  t = opaque_tid();
  for (int i0 = 0; i0 < NKO; i0 += CKO) {
    double la[CKO], lb[CKO];
    double2 dd[CKO], cc[CKO];
#pragma unroll
    for (int c = 0; c < CKO; ++c) {
      const int k = t + RL_THREADS * (i0 + c);
      if (i0 + c < NKO && k < h / 2) {
        la[c] = lam[2 * k + 1];
        lb[c] = lam[2 * k + 2 * h + 1];
        dd[c] = wm(2 * k + 1);
        cc[c] = wm(2 * k);
      }
    }
#pragma unroll
    for (int c = 0; c < CKO; ++c) {
      const int k = t + RL_THREADS * (i0 + c);
      if (!(i0 + c < NKO && k < h / 2)) continue;
      const int kr = h - 1 - k;
      double2 gk, gr;
      rl_odd_pair(X[lpad(k)], X[lpad(kr)], la[c], lb[c], dd[c], cc[c], om, gk, gr);
      X[lpad(k)] = gk;
      X[lpad(kr)] = gr;
    }
  }
  __syncthreads();
  rl_fft<LH>(X, ptw);
  // tO_{2p} + i tO_{2p+1} = conj(w_m^{2p} X[p]); C y0 = tE / m + tO / m
  t = opaque_tid();
#pragma unroll
  for (int i0 = 0; i0 < NI; i0 += CF) {
    int32_t r[CF][2];
    double hv[CF][2], yv[CF][2];
    double2 wp[CF];
#pragma unroll
    for (int c = 0; c < CF; ++c) rows(i0 + c, r[c]);
#pragma unroll
    for (int c = 0; c < CF; ++c) {
      if (!in_pos(i0 + c)) continue;
      const int jj = 2 * (t + RL_THREADS * (i0 + c));
      wp[c] = wm(jj);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        hv[c][u] = r[c][u] >= 0 ? hrow[jj + u] : 0.0;
        yv[c][u] = r[c][u] >= 0 ? ydp[jj + u] : 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < CF; ++c) {
      if (!in_pos(i0 + c)) continue;
      const double2 gz = conj2(cmul(wp[c], X[lpad(t + RL_THREADS * (i0 + c))]));
      const double2 tv = te[i0 + c];
      const fv2 yy = yk[i0 + c];
      double ov[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const double cz = (u ? tv.y : tv.x) + (u ? gz.y : gz.x) * inv_m;
        const float yf = u ? yy.y : yy.x;
        const double xd = isfinite(yf) ? (double)yf : 0.0;
        ov[u] = hv[c][u] - cz;
        if (r[c][u] < 0) continue;
        a.hy += hv[c][u] * xd;
        a.ydh += hv[c][u] * yv[c][u];
        a.yc += xd * cz;
      }
      es.pair(r[c], ov[0], ov[1]);
    }
  }
  __syncthreads();
  acc.hy += a.hy;
  acc.ydh += a.ydh;
  acc.yc += a.yc;
  acc.bad += a.bad;
}

// Segments whose packed h-point DFTs (h = 2 hh, hh = 2^(LH-1) the largest in-LDS length)
// exceed the LDS array.  Each h-point forward DFT is two hh-point DFTs, of the even- and
// odd-indexed packed samples (Z_k = E_k + w_h^k O_k, Z_{k+hh} = E_k - w_h^k O_k); E waits
// in registers while O is transformed in LDS.  The pointwise stage works on quadruples of
// frequencies {k, k2, k + hh, k2 + hh}, k < hh/2, closed under both its pairing and the
// split (k2 = hh - k for the even part, hh - 1 - k for the odd part), and returns the two
// halves of the next DFT's input (decimation in frequency): A_k = G_k + G_{k+hh}, whose
// hh-point DFT gives outputs 2n, and B_k = (G_k - G_{k+hh}) w_h^k, outputs 2n + 1.  A is
// written over O in LDS and B waits in the registers E held.  Output 2n + s carries the
// samples 4n + 2s and 4n + 2s + 1, so a thread owns the same samples in every phase.
//
// The caller supplies the data and takes the results:
//   stage(s, odd)  writes X[n] = x_{4n+2s} + i x_{4n+2s+1} for n < hh (times w_m^{4n+2s}
//                  in the odd part) and ends with a barrier;
//   mult(r)        the multiplier of frequency r < m (real eigenvalue or complex spectrum);
//   emit(s, odd)   reads X[n], n < hh, after the last DFT of half s: t_{2p} + i t_{2p+1} =
//                  conj(X[n]) (even part) or conj(w_m^{2p} X[n]) (odd part), p = 2n + s,
//                  with C x = (t_even + t_odd) / m.
// The thread index is re-read (opaquely) at each phase, so that per-position addresses and
// masks are recomputed there instead of being held in registers across phases.
template <int LH, class Stage, class Mult, class Emit>
__device__ __forceinline__ void rl_split_parts(double2 *X, const gmem<const dv2> *__restrict__ tw,
                                               const gmem<const dv2> *__restrict__ ptw, Stage &&stage,
                                               Mult &&mult, Emit &&emit) {
  constexpr int LHH = LH - 1;
  constexpr int h = 1 << LH, hh = 1 << LHH;
  static_assert(hh >= 2 * RL_THREADS && hh % (2 * RL_THREADS) == 0, "whole quadruples per thread");
  constexpr int NQ = hh / 2 / RL_THREADS;  // quadruples per thread
  auto wm = [&](int r) {  // w_m^r, 0 <= r < m
    const dv2 v = tw[r];
    return make_double2(v.x, -v.y);
  };
  int t = opaque_tid();
#pragma unroll 1
  for (int part = 0; part < 2; ++part) {
    const bool odd = part == 1;
    // quadruple i of this thread: k = t + RL_THREADS i and its partner k2; the even part's
    // k = hh/2 (its own partner) goes to thread 0 as an extra quadruple
    auto k_of = [&](int i) { return i < NQ ? t + RL_THREADS * i : hh / 2; };
    auto k2_of = [&](int k) { return odd ? hh - 1 - k : (hh - k) & (hh - 1); };
    const bool extra = !odd && t == 0;
    double2 ra[NQ + 1], rb[NQ + 1];  // E_k, E_k2, then B_k, B_k2
    stage(0, odd);
    rl_fft<LHH>(X, ptw);
    t = opaque_tid();
#pragma unroll
    for (int i = 0; i <= NQ; ++i) {
      if (i == NQ && !extra) continue;
      const int k = k_of(i);
      ra[i] = X[lpad(k)];
      rb[i] = X[lpad(k2_of(k))];
    }
    __syncthreads();
    stage(1, odd);
    rl_fft<LHH>(X, ptw);
    t = opaque_tid();
#pragma unroll
    for (int i = 0; i <= NQ; ++i) {
      if (i == NQ && !extra) continue;
      const int k = k_of(i), k2 = k2_of(k);
      const double2 wk = wm(4 * k), wk2 = wm(4 * k2);  // w_h^k, w_h^k2
      const double2 ok = cmul(wk, X[lpad(k)]), ok2 = cmul(wk2, X[lpad(k2)]);
      const double2 zk = cadd(ra[i], ok), zkh = csub(ra[i], ok);     // Z_k, Z_{k+hh}
      const double2 zk2 = cadd(rb[i], ok2), zk2h = csub(rb[i], ok2); // Z_k2, Z_{k2+hh}
      double2 gk, gkh, gk2 = zk2, gk2h = zk2h, unused;
      if (!odd) {
        if (k == 0) {  // self-paired 0 and hh
          rl_even_pair(zk, zk, mult(0), mult(2 * h), wm(0), gk, unused);
          rl_even_pair(zkh, zkh, mult(h), mult(h), wm(h), gkh, unused);
        } else {
          // pairs (k, h - k = k2 + hh) and (k2, h - k2 = k + hh)
          rl_even_pair(zk, zk2h, mult(2 * k), mult(2 * h - 2 * k), wm(2 * k), gk, gk2h);
          rl_even_pair(zk2, zkh, mult(2 * k2), mult(2 * h - 2 * k2), wm(2 * k2), gk2, gkh);
        }
      } else {
        // pairs (k, h - 1 - k = k2 + hh) and (k2, h - 1 - k2 = k + hh)
        const double2 om = wm(1);
        rl_odd_pair(zk, zk2h, mult(2 * k + 1), mult(2 * k + 2 * h + 1), wm(2 * k + 1), wm(2 * k),
                    om, gk, gk2h);
        rl_odd_pair(zk2, zkh, mult(2 * k2 + 1), mult(2 * k2 + 2 * h + 1), wm(2 * k2 + 1),
                    wm(2 * k2), om, gk2, gkh);
      }
      X[lpad(k)] = cadd(gk, gkh);
      ra[i] = cmul(csub(gk, gkh), wk);
      if (k2 != k) {
        X[lpad(k2)] = cadd(gk2, gk2h);
        rb[i] = cmul(csub(gk2, gk2h), wk2);
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      t = opaque_tid();
      if (s == 1) {
#pragma unroll
        for (int i = 0; i <= NQ; ++i) {
          if (i == NQ && !extra) continue;
          const int k = k_of(i), k2 = k2_of(k);
          X[lpad(k)] = ra[i];
          if (k2 != k) X[lpad(k2)] = rb[i];
        }
        __syncthreads();
      }
      rl_fft<LHH>(X, ptw);
      emit(s, odd);
      __syncthreads();
    }
  }
}

// Segments with m = 16 hq (h = 4 hq, hq = 2^(LH-2) the largest in-LDS length): each
// h-point DFT is four hq-point DFTs of the packed samples p = 4q + s (radix-4 decimation
// in time): Z_{k0 + hq j} = sum_s (-i)^{sj} U_s with U_s = w_h^{s k0} F_s[k0].  F_0..F_2
// wait in the workgroup's global scratch S (3 hq complex) while F_3 is in LDS.  The
// pointwise stage takes the frequencies in groups {k0, k1} x {j = 0..3}, k1 = hq - k0
// (even part) or hq - 1 - k0 (odd part), closed under its pairing (partner of k0 + hq j
// is k1 + hq (3 - j)); a group yields the four quarters of the next DFT's input (radix-4
// decimation in frequency), A_s[p0] = w_h^{s p0} sum_j (-i)^{sj} G[p0 + hq j], whose
// hq-point DFTs give the outputs 4n + s.  A_3 goes to LDS, A_0..A_2 over F_0..F_2 in S.
// Callbacks as for rl_split_parts, with quarters s = 0..3 (samples 8n + 2s, 8n + 2s + 1).

// V_j = sum_s (-i)^{sj} U_s (4-point forward DFT)
__device__ __forceinline__ void dft4(const double2 (&u)[4], double2 (&v)[4]) {
  const double2 a = cadd(u[0], u[2]), b = csub(u[0], u[2]);
  const double2 c = cadd(u[1], u[3]), d = csub(u[1], u[3]);
  const double2 md = make_double2(d.y, -d.x);  // -i d
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, md);
  v[3] = csub(b, md);
}

template <int LH, class Stage, class Mult, class Emit>
__device__ __forceinline__ void rl_quad_parts(double2 *X, gmem<dv2> *__restrict__ S,
                                              const gmem<const dv2> *__restrict__ tw,
                                              const gmem<const dv2> *__restrict__ ptw, Stage &&stage,
                                              Mult &&mult, Emit &&emit) {
  constexpr int LHQ = LH - 2;
  constexpr int h = 1 << LH, hq = 1 << LHQ;
  static_assert(hq >= 2 * RL_THREADS && hq % (2 * RL_THREADS) == 0, "whole groups per thread");
  constexpr int NI = hq / RL_THREADS;      // positions per thread and quarter
  constexpr int NG = hq / 2 / RL_THREADS;  // groups per thread
  auto wm = [&](int r) {  // w_m^r, 0 <= r < m
    const dv2 v = tw[r];
    return make_double2(v.x, -v.y);
  };
  int t = opaque_tid();
#pragma unroll 1
  for (int part = 0; part < 2; ++part) {
    const bool odd = part == 1;
#pragma unroll 1
    for (int s = 0; s < 4; ++s) {
      stage(s, odd);
      rl_fft<LHQ>(X, ptw);
      if (s < 3) {
        t = opaque_tid();
        for (int i = 0; i < NI; ++i) {
          const int n = t + RL_THREADS * i;
          S[s * hq + n] = to_dv2(X[lpad(n)]);
        }
        __syncthreads();
      }
    }
    t = opaque_tid();
    // the even part's k0 = hq/2 (its own partner) goes to thread 0 as an extra group
#pragma unroll 1
    for (int i = 0; i <= NG; ++i) {
      if (i == NG && (odd || t != 0)) continue;
      const int k0 = i < NG ? t + RL_THREADS * i : hq / 2;
      const int k1 = odd ? hq - 1 - k0 : (hq - k0) & (hq - 1);
      double2 za[4], zb[4], ga[4], gb[4];
      {
        double2 u[4];
#pragma unroll
        for (int q = 0; q < 3; ++q) u[q] = from_dv2(S[q * hq + k0]);
        u[3] = X[lpad(k0)];
#pragma unroll
        for (int q = 1; q < 4; ++q) u[q] = cmul(wm(4 * q * k0), u[q]);
        dft4(u, za);
#pragma unroll
        for (int q = 0; q < 3; ++q) u[q] = from_dv2(S[q * hq + k1]);
        u[3] = X[lpad(k1)];
#pragma unroll
        for (int q = 1; q < 4; ++q) u[q] = cmul(wm(4 * q * k1), u[q]);
        dft4(u, zb);
      }
      if (!odd && k0 == 0) {
        // 0 and h/2 pair with themselves, hq with 3 hq
        double2 unused;
        rl_even_pair(za[0], za[0], mult(0), mult(2 * h), wm(0), ga[0], unused);
        rl_even_pair(za[1], za[3], mult(2 * hq), mult(2 * h - 2 * hq), wm(2 * hq), ga[1], ga[3]);
        rl_even_pair(za[2], za[2], mult(h), mult(h), wm(h), ga[2], unused);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = k0 + hq * j;  // partner h - k (even) or h - 1 - k (odd) = k1 + hq (3 - j)
          if (!odd)
            rl_even_pair(za[j], zb[3 - j], mult(2 * k), mult(2 * h - 2 * k), wm(2 * k), ga[j],
                         gb[3 - j]);
          else
            rl_odd_pair(za[j], zb[3 - j], mult(2 * k + 1), mult(2 * k + 2 * h + 1), wm(2 * k + 1),
                        wm(2 * k), wm(1), ga[j], gb[3 - j]);
        }
      }
      // quarters of the inverse DFT's input at p0 = k0 and p0 = k1
      double2 v[4];
      dft4(ga, v);
      X[lpad(k0)] = cmul(wm(12 * k0), v[3]);
#pragma unroll
      for (int q = 0; q < 3; ++q) S[q * hq + k0] = to_dv2(q ? cmul(wm(4 * q * k0), v[q]) : v[q]);
      if (k1 != k0) {
        dft4(gb, v);
        X[lpad(k1)] = cmul(wm(12 * k1), v[3]);
#pragma unroll
        for (int q = 0; q < 3; ++q) S[q * hq + k1] = to_dv2(q ? cmul(wm(4 * q * k1), v[q]) : v[q]);
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int s = 3; s >= 0; --s) {
      if (s < 3) {
        t = opaque_tid();
        for (int i = 0; i < NI; ++i) {
          const int n = t + RL_THREADS * i;
          X[lpad(n)] = from_dv2(S[s * hq + n]);
        }
        __syncthreads();
      }
      rl_fft<LHQ>(X, ptw);
      emit(s, odd);
      __syncthreads();
    }
  }
}

// Refinement of one template over a segment whose transforms split into P = 2 halves
// (m = 8 hh, rl_split_parts) or P = 4 quarters (m = 16 hq, rl_quad_parts, with the
// workgroup's scratch S): part s of a transform carries the samples 2 P n + 2 s and
// 2 P n + 2 s + 1.
template <int LH, int P>
__device__ __noinline__ void rl_segment_split(const RefItem &it, const SegDev &sd, int64_t b,
                                              double2 *X, gmem<dv2> *S_, RlAcc &acc) {
  gmem<dv2> *S = uni(S_);
  static_assert(P == 2 || P == 4, "halves or quarters");
  constexpr int h = 1 << LH;
  constexpr int NI = h / P / RL_THREADS;  // position iterations per part
  constexpr int CH = NI < RL_CH ? NI : RL_CH;  // positions per batch of memory accesses
  static_assert(NI % CH == 0, "whole chunks");
  int t = opaque_tid();
  const gmem<const float> *__restrict__ y = gpu(it.y0 + b * it.n_pad);
  const gmem<const double> *__restrict__ hrow = gpu(template_row(it, b) + sd.offset);
  const gmem<const double> *__restrict__ ydp = gpu(it.yd_pos + sd.offset);
  const gmem<const int32_t> *__restrict__ p2r = gpu(it.pos2row + sd.offset);
  gmem<double> *__restrict__ e = gpu(it.e64 + b * it.n_pad);  // t_E / m between the parts
  const EsOut es(it.es_hi, it.es_lo, it.tks, b);
  const gmem<const dv2> *__restrict__ tw = gpu((const dv2 *)sd.tw);  // (cos, sin) of 2 pi r / m
  const gmem<const dv2> *__restrict__ ptw = gpu((const dv2 *)sd.ptw);  // passes of the part DFTs
  const gmem<const double> *__restrict__ lam = gpu(sd.lam);
  const int len = uni((int)sd.length);
  const bool dense = uni((int)(sd.nkeep == sd.length)) != 0;
  const int32_t row0 = uni((int32_t)sd.row0);
  const double inv_m = 1.0 / (double)(4 * h);
  RlAcc a{0, 0, 0, 0};  // added to the caller's sums at the end
  auto wm = [&](int r) {  // w_m^r, 0 <= r < m
    const dv2 v = tw[r];
    return make_double2(v.x, -v.y);
  };
  auto row_of = [&](int jj) -> int32_t {
    if (jj >= len) return -1;
    return dense ? row0 + jj : p2r[jj];
  };
  auto finite_or_flag = [&](float v) -> double {
    if (!isfinite(v)) {
      a.bad = 1.0;
      return 0.0;
    }
    return (double)v;
  };
  // rows and y0 values of the samples 2Pn + 2s, 2Pn + 2s + 1, n = t + RL_THREADS (i0 + c)
  auto load_x = [&](int i0, int s, int32_t (&rr)[CH][2], float (&xv)[CH][2]) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int n = t + RL_THREADS * (i0 + c);
      rr[c][0] = row_of(2 * P * n + 2 * s);
      rr[c][1] = row_of(2 * P * n + 2 * s + 1);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int u = 0; u < 2; ++u) xv[c][u] = rr[c][u] >= 0 ? y[rr[c][u]] : 0.f;
  };
  auto stage = [&](int s, bool odd) {
    t = opaque_tid();
    for (int i0 = 0; i0 < NI; i0 += CH) {
      int32_t rr[CH][2];
      float xv[CH][2];
      load_x(i0, s, rr, xv);
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int n = t + RL_THREADS * (i0 + c);
        const double2 z = make_double2(finite_or_flag(xv[c][0]), finite_or_flag(xv[c][1]));
        X[lpad(n)] = odd ? cmul(z, wm(2 * P * n + 2 * s)) : z;
      }
    }
    __syncthreads();
  };
  auto mult = [&](int r) { return lam[r]; };
  // even part: t_E / m parked in e; odd part: C y0 = e + t_O / m, then the residual
  // h - C y0 (written split) and the dot products
  auto emit = [&](int s, bool odd) {
    t = opaque_tid();
    for (int i0 = 0; i0 < NI; i0 += CH) {
      int32_t rr[CH][2];
      float xv[CH][2];
      if (!odd) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int n = t + RL_THREADS * (i0 + c);
          rr[c][0] = row_of(2 * P * n + 2 * s);
          rr[c][1] = row_of(2 * P * n + 2 * s + 1);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const double2 v = X[lpad(t + RL_THREADS * (i0 + c))];
          if (rr[c][0] >= 0) e[rr[c][0]] = v.x * inv_m;
          if (rr[c][1] >= 0) e[rr[c][1]] = -v.y * inv_m;
        }
        continue;
      }
      double ev[CH][2], hv[CH][2], yv[CH][2];
      load_x(i0, s, rr, xv);
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int n = t + RL_THREADS * (i0 + c);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int jj = 2 * P * n + 2 * s + u;
          ev[c][u] = rr[c][u] >= 0 ? e[rr[c][u]] : 0.0;
          hv[c][u] = rr[c][u] >= 0 ? hrow[jj] : 0.0;
          yv[c][u] = rr[c][u] >= 0 ? ydp[jj] : 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int n = t + RL_THREADS * (i0 + c);
        const double2 gz = conj2(cmul(wm(2 * P * n + 2 * s), X[lpad(n)]));
        double ov[2] = {0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (rr[c][u] < 0) continue;
          const double cz = ev[c][u] + (u ? gz.y : gz.x) * inv_m;
          const double xd = isfinite(xv[c][u]) ? (double)xv[c][u] : 0.0;
          ov[u] = hv[c][u] - cz;
          a.hy += hv[c][u] * xd;
          a.ydh += hv[c][u] * yv[c][u];
          a.yc += xd * cz;
        }
        es.pair(rr[c], ov[0], ov[1]);
      }
    }
  };

  for (int64_t q = sd.row0 + sd.nkeep + t; q < sd.row0 + sd.npad; q += RL_THREADS)
    es.put((int32_t)q, 0.0);
  if constexpr (P == 2)
    rl_split_parts<LH>(X, tw, ptw, stage, mult, emit);
  else
    rl_quad_parts<LH>(X, S, tw, ptw, stage, mult, emit);
  acc.hy += a.hy;
  acc.ydh += a.ydh;
  acc.yc += a.yc;
  acc.bad += a.bad;
}

// Work entry: (item, template), item -1 for padding.  Persistent grid, one workgroup per CU
// (the LDS array).  Segments of the largest circulant length also need scratch: 3 x 8192
// complex doubles per workgroup at qscratch (NULL when the launch has none).
__global__ __launch_bounds__(RL_THREADS) void k_refine_lds(const RefItem *__restrict__ items,
                                                           const int2 *__restrict__ work,
                                                           int64_t n_work,
                                                           double2 *__restrict__ qscratch) {
  extern __shared__ double2 rl_smem[];
  double2 *X = rl_smem;
  double *red = (double *)(rl_smem + RL_XN);
  gmem<dv2> *S = qscratch ? gpu((dv2 *)(qscratch + (int64_t)blockIdx.x * RL_QUAD_SCRATCH)) : nullptr;
  for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
    const int2 wk = work[wi];
    if (wk.x < 0) continue;  // padding of the work list
    const RefItem &it = items[wk.x];
    const int64_t b = wk.y;
    RlAcc acc{0, 0, 0, 0};
    for (int sg = 0; sg < it.n_segs; ++sg) {
      const SegDev sd = it.segs[sg];
      switch (sd.log2m - 2) {
#define TDA_RL(LH) \
  case LH: rl_segment<LH>(it, sd, b, X, acc); break;
        TDA_RL(2) TDA_RL(3) TDA_RL(4) TDA_RL(5) TDA_RL(6) TDA_RL(7) TDA_RL(8) TDA_RL(9)
        TDA_RL(10) TDA_RL(11) TDA_RL(12) TDA_RL(13)
#undef TDA_RL
        case RL_LHMAX + 1: rl_segment_split<RL_LHMAX + 1, 2>(it, sd, b, X, nullptr, acc); break;
        case RL_LHMAX + 2:
          if (S) rl_segment_split<RL_LHMAX + 2, 4>(it, sd, b, X, S, acc);
          else acc.bad = 1.0;
          break;
        default: acc.bad = 1.0;
      }
    }
    double sums[4] = {acc.hy, acc.ydh, acc.yc, acc.bad};
    block_sum0(sums, red);
    if (threadIdx.x == 0) {
      const double s_hy = sums[0], s_ydh = sums[1], s_yc = sums[2], s_bad = sums[3];
      const double nan = __builtin_nan("");
      it.qpart[b] = s_bad > 0 ? nan : it.qdd[0] - 2.0 * s_ydh + 2.0 * s_hy - s_yc;
      if (it.dh_out) it.dh_out[b] = s_bad > 0 || isnan(it.qdd[0]) ? nan : s_ydh;
      if (it.hh_out) it.hh_out[b] = s_bad > 0 ? nan : 2.0 * s_hy - s_yc;
    }
  }
}


hipError_t launch_refine_lds(const RefItem *items, const int2 *work, int64_t n_work,
                             double *qscratch, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>(n_work, qscratch ? RL_QUAD_WG : 2048);
  hipLaunchKernelGGL(k_refine_lds, dim3((unsigned)g), dim3(RL_THREADS), RL_LDS_BYTES, s, items,
                     work, n_work, (double2 *)qscratch);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Gohberg-Semencul path
// For a segment without excluded samples C is symmetric Toeplitz.  With x = C^-1 e_1
// (x_0 > 0) the inverse is (1/x_0) (L(x) L(x)^T - L(z) L(z)^T), z = (0, x_{n-1}, ..., x_1),
// L(v) the lower-triangular Toeplitz matrix with first column v (Sec. III.A.3), so
//   q = r^T C^-1 r = (||L(x)^T r||^2 - ||L(z)^T r||^2) / x_0,
// each L(v)^T r a correlation, i.e. the first n outputs of the circulant product with
// multiplier conj(DFT_m(v)) (m >= 2n, zero padding), computed with the in-LDS parity split
// of the refinement (complex multipliers of real sequences keep the pairing identities).
// x and log det C come from Levinson-Durbin.

// Durbin's recursion: a = (1, a_1, .., a_k) the order-k prediction-error filter, E_k its
// error energy; reflection kappa_k = -(sum_{j<k} a_j acf[k - j]) / E_{k-1}, a_j += kappa_k
// a_{k-j} (pairwise, in place), E_k = E_{k-1} (1 - kappa_k^2); x = a / E_{n-1}.
// The coefficients live in LDS, or (kGlobal, for n beyond the LDS) in x itself; either
// way only this workgroup touches them, and its barriers order the accesses.
template <bool kGlobal>
__global__ __launch_bounds__(1024) void k_levinson(const double *__restrict__ acf, int n,
                                                   double *__restrict__ x,
                                                   double *__restrict__ logdet_out,
                                                   int32_t *__restrict__ fail) {
  extern __shared__ double lev_lds[];  // [n] unless kGlobal
  double *lev_a = kGlobal ? x : lev_lds;
  __shared__ double wsum[16];
  __shared__ double shE, shL;
  __shared__ int shFail;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int j = t; j < n; j += 1024) lev_a[j] = j == 0 ? 1.0 : 0.0;
  if (t == 0) {
    shE = acf[0];
    shL = log(acf[0]);
    shFail = (acf[0] > 0.0 && isfinite(acf[0])) ? -1 : 0;
  }
  __syncthreads();
  for (int k = 1; k < n && shFail < 0; ++k) {
    double part = 0.0;
    for (int j = t; j < k; j += 1024) part += lev_a[j] * acf[k - j];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) wsum[wv] = part;
    __syncthreads();
    double num = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) num += wsum[w];
    const double kappa = -num / shE;
    for (int j = t; 2 * j <= k; j += 1024) {
      const double aj = lev_a[j], ak = lev_a[k - j];
      if (2 * j == k) {
        lev_a[j] = aj + kappa * aj;
      } else {
        lev_a[j] = aj + kappa * ak;
        lev_a[k - j] = ak + kappa * aj;
      }
    }
    __syncthreads();
    if (t == 0) {
      const double E = shE * (1.0 - kappa * kappa);
      if (!(E > 0.0) || !isfinite(E)) {
        shFail = k;
      } else {
        shE = E;
        shL += log(E);
      }
    }
    __syncthreads();
  }
  for (int j = t; j < n; j += 1024) x[j] = lev_a[j] / shE;
  if (t == 0) {
    *logdet_out = shL;
    *fail = shFail;
  }
}

hipError_t launch_levinson(const double *acf, int64_t n, double *x, double *logdet,
                           int32_t *fail, hipStream_t s) {
  if (n < 1 || n > GS_MAX_LEN) return hipErrorInvalidValue;
  if (n <= RL_MAX_LEV)
    hipLaunchKernelGGL(k_levinson<false>, dim3(1), dim3(1024), (size_t)n * sizeof(double), s, acf,
                       (int)n, x, logdet, fail);
  else
    hipLaunchKernelGGL(k_levinson<true>, dim3(1), dim3(1024), 0, s, acf, (int)n, x, logdet, fail);
  return hipGetLastError();
}

// M_k = sum_j v_j exp(+2 pi i j k / m) = conj(DFT_m(v))_k, direct sums in FP64
__global__ void k_gs_spectra(const double *__restrict__ x, int64_t n, int64_t m,
                             const double *__restrict__ tw, double *__restrict__ M1,
                             double *__restrict__ M2) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= m) return;
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
  int64_t r = 0;  // j k mod m
  for (int64_t j = 0; j < n; ++j) {
    const double c = tw[2 * r], sn = tw[2 * r + 1];
    const double xv = x[j], zv = j == 0 ? 0.0 : x[n - j];
    ar += xv * c;
    ai += xv * sn;
    br += zv * c;
    bi += zv * sn;
    r += k;
    if (r >= m) r -= m;
  }
  M1[2 * k] = ar;
  M1[2 * k + 1] = ai;
  M2[2 * k] = br;
  M2[2 * k + 1] = bi;
}

hipError_t launch_gs_spectra(const double *x, int64_t n, int64_t m, const double *tw,
                             double *M1, double *M2, hipStream_t s) {
  hipLaunchKernelGGL(k_gs_spectra, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, x, n, m,
                     tw, M1, M2);
  return hipGetLastError();
}

// Sums over this thread's outputs j < length of (L(v)^T r)_j^2 for the two generators
// v = x (multiplier M1 = conj(DFT_m(x))) and v = z (M2); returns the first minus the
// second.  Both products start from the same transform of the residual, so each part
// (circulant, skew-circulant) takes one forward DFT and two inverse ones: the pointwise
// stage writes the first product's input to LDS and keeps the second's in registers until
// the first has been transformed back.  The first product's circulant output waits in the
// workgroup's scratch at tes, the second's at tes2.
template <int LH>
__device__ __noinline__ double gs_pair(const GsItem &it, const GsSeg &sd, int64_t b,
                                       const gmem<const dv2> *__restrict__ M1_,
                                       const gmem<const dv2> *__restrict__ M2_, double2 *X,
                                       gmem<double> *__restrict__ tes_) {
  constexpr int h = 1 << LH;
  constexpr int NI = h >= RL_THREADS ? h / RL_THREADS : 1;
  constexpr int NKE = (h / 2 + RL_THREADS) / RL_THREADS;
  constexpr int NKO = h / 2 >= RL_THREADS ? h / 2 / RL_THREADS : 1;
  constexpr int CL = NI < RL_CHL ? NI : RL_CHL;
  constexpr int CK = 3;  // frequency pairs per batch of multiplier loads
  const gmem<const dv2> *__restrict__ M1 = uni(M1_);
  const gmem<const dv2> *__restrict__ M2 = uni(M2_);
  gmem<double> *__restrict__ tes = uni(tes_);
  const gmem<const double> *__restrict__ hrow = gpu(gs_template_row(it, b) + sd.offset);
  const gmem<const double> *__restrict__ dd = gpu(it.d + sd.offset);
  const gmem<const dv2> *__restrict__ tw = gpu((const dv2 *)sd.tw);
  const gmem<const dv2> *__restrict__ ptw = gpu((const dv2 *)sd.ptw);
  const int len = uni((int)sd.length);
  gmem<double> *__restrict__ tes2 = tes + ((len + 1) & ~1);
  const double inv_m = 1.0 / (double)(4 * h);
  // the thread index is re-read (opaquely) at each phase, so that per-position addresses
  // and masks are recomputed there rather than held in registers across phases
  int t = opaque_tid();
  auto wm = [&](int r) {
    const dv2 v = tw[r];
    return make_double2(v.x, -v.y);
  };
  auto in_pos = [&](int i) { return i < NI && t + RL_THREADS * i < h; };
  // residual samples 2p, 2p + 1 into X (times w_m^{2p} for the skew-circulant part)
  auto stage = [&](bool odd) {
    t = opaque_tid();
    for (int i0 = 0; i0 < NI; i0 += CL) {
      double rv[CL][2];
      double2 wp[CL];
#pragma unroll
      for (int c = 0; c < CL; ++c) {
        const int jj = 2 * (t + RL_THREADS * (i0 + c));
#pragma unroll
        for (int u = 0; u < 2; ++u)
          rv[c][u] = (in_pos(i0 + c) && jj + u < len) ? dd[jj + u] - hrow[jj + u] : 0.0;
        if (odd && in_pos(i0 + c)) wp[c] = wm(jj);
      }
#pragma unroll
      for (int c = 0; c < CL; ++c) {
        if (!in_pos(i0 + c)) continue;
        const double2 z = make_double2(rv[c][0], rv[c][1]);
        X[lpad(t + RL_THREADS * (i0 + c))] = odd ? cmul(z, wp[c]) : z;
      }
    }
    __syncthreads();
  };
  // the second product's input, written by the thread that computed it
  constexpr int NG = ((NKE > NKO ? NKE : NKO) + CK - 1) / CK * CK;
  double2 g2k[NG], g2r[NG];
  auto second_to_lds = [&](auto odd_c) {
    constexpr bool odd = decltype(odd_c)::value;
    t = opaque_tid();
#pragma unroll
    for (int c = 0; c < (odd ? NKO : NKE); ++c) {
      const int k = t + RL_THREADS * c;
      if (odd ? !(k < h / 2) : !(k <= h / 2)) continue;
      const int kr = odd ? h - 1 - k : (h - k) & (h - 1);
      X[lpad(k)] = g2k[c];
      if (odd || (k != 0 && k != h / 2)) X[lpad(kr)] = g2r[c];
    }
    __syncthreads();
  };

  // ---- even frequencies
  stage(false);
  rl_fft<LH>(X, ptw);
  t = opaque_tid();
#pragma unroll
  for (int i0 = 0; i0 < NKE; i0 += CK) {
    double2 m1a[CK], m1b[CK], m2a[CK], m2b[CK], cc[CK];
#pragma unroll
    for (int c = 0; c < CK; ++c) {
      const int k = t + RL_THREADS * (i0 + c);
      if (i0 + c < NKE && k <= h / 2) {
        m1a[c] = from_dv2(M1[2 * k]);
        m1b[c] = from_dv2(M1[2 * h - 2 * k]);
        m2a[c] = from_dv2(M2[2 * k]);
        m2b[c] = from_dv2(M2[2 * h - 2 * k]);
        cc[c] = wm(2 * k);
      }
    }
#pragma unroll
    for (int c = 0; c < CK; ++c) {
      const int k = t + RL_THREADS * (i0 + c);
      if (!(i0 + c < NKE && k <= h / 2)) continue;
      const int kr = (h - k) & (h - 1);
      const double2 vk = X[lpad(k)], vr = X[lpad(kr)];
      double2 gk, gr;
      rl_even_pair(vk, vr, m1a[c], m1b[c], cc[c], gk, gr);
      rl_even_pair(vk, vr, m2a[c], m2b[c], cc[c], g2k[i0 + c], g2r[i0 + c]);
      X[lpad(k)] = gk;
      if (k != 0 && k != h / 2) X[lpad(kr)] = gr;
    }
  }
  __syncthreads();
  // the even part of outputs 2p, 2p + 1 of each product waits in scratch (same thread later)
  auto park = [&](gmem<double> *dst) {
    t = opaque_tid();
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int p = t + RL_THREADS * i;
      if (!in_pos(i) || 2 * p >= len) continue;
      const double2 g = X[lpad(p)];
      dst[2 * p] = g.x;
      if (2 * p + 1 < len) dst[2 * p + 1] = -g.y;
    }
    __syncthreads();
  };
  rl_fft<LH>(X, ptw);
  park(tes);
  second_to_lds(std::false_type{});
  rl_fft<LH>(X, ptw);
  park(tes2);

  // ---- odd frequencies
  stage(true);
  rl_fft<LH>(X, ptw);
  t = opaque_tid();
  const double2 om = wm(1);
#pragma unroll
  for (int i0 = 0; i0 < NKO; i0 += CK) {
    double2 m1a[CK], m1b[CK], m2a[CK], m2b[CK], dv[CK], cc[CK];
#pragma unroll
    for (int c = 0; c < CK; ++c) {
      const int k = t + RL_THREADS * (i0 + c);
      if (i0 + c < NKO && k < h / 2) {
        m1a[c] = from_dv2(M1[2 * k + 1]);
        m1b[c] = from_dv2(M1[2 * k + 2 * h + 1]);
        m2a[c] = from_dv2(M2[2 * k + 1]);
        m2b[c] = from_dv2(M2[2 * k + 2 * h + 1]);
        dv[c] = wm(2 * k + 1);
        cc[c] = wm(2 * k);
      }
    }
#pragma unroll
    for (int c = 0; c < CK; ++c) {
      const int k = t + RL_THREADS * (i0 + c);
      if (!(i0 + c < NKO && k < h / 2)) continue;
      const int kr = h - 1 - k;
      const double2 vk = X[lpad(k)], vr = X[lpad(kr)];
      double2 gk, gr;
      rl_odd_pair(vk, vr, m1a[c], m1b[c], dv[c], cc[c], om, gk, gr);
      rl_odd_pair(vk, vr, m2a[c], m2b[c], dv[c], cc[c], om, g2k[i0 + c], g2r[i0 + c]);
      X[lpad(k)] = gk;
      X[lpad(kr)] = gr;
    }
  }
  __syncthreads();
  // outputs (tE + tO) / m of one product, squared and summed
  auto sumsq = [&](const gmem<double> *src) {
    t = opaque_tid();
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int p = t + RL_THREADS * i;
      if (!in_pos(i) || 2 * p >= len) continue;
      const double2 gz = conj2(cmul(wm(2 * p), X[lpad(p)]));
      const double c0 = (src[2 * p] + gz.x) * inv_m;
      ss += c0 * c0;
      if (2 * p + 1 < len) {
        const double c1 = (src[2 * p + 1] + gz.y) * inv_m;
        ss += c1 * c1;
      }
    }
    __syncthreads();
    return ss;
  };
  rl_fft<LH>(X, ptw);
  const double s1 = sumsq(tes);
  second_to_lds(std::true_type{});
  rl_fft<LH>(X, ptw);
  const double s2 = sumsq(tes2);
  return s1 - s2;
}

// One correlation's sum over this thread's outputs j < length of (L(v)^T r)_j^2
// (multiplier M), for segments whose transforms split in P = 2 halves (m = 8 hh) or P = 4
// quarters (m = 16 hq, with the workgroup's scratch S), through the drivers of the
// refinement.  The two correlations run one after the other here: the split drivers
// already hold half of each transform in registers.
template <int LH, int P>
__device__ __noinline__ double gs_sumsq_split(const GsItem &it, const GsSeg &sd, int64_t b,
                                              const gmem<const dv2> *__restrict__ M_, double2 *X,
                                              gmem<dv2> *S_, gmem<double> *__restrict__ tes_) {
  const gmem<const dv2> *__restrict__ M = uni(M_);
  gmem<dv2> *S = uni(S_);
  gmem<double> *__restrict__ tes = uni(tes_);
  static_assert(P == 2 || P == 4, "halves or quarters");
  constexpr int h = 1 << LH;
  constexpr int NI = h / P / RL_THREADS;
  static_assert(NI % RL_CH == 0, "whole chunks");
  int t = opaque_tid();
  const gmem<const double> *__restrict__ hrow = gpu(gs_template_row(it, b) + sd.offset);
  const gmem<const double> *__restrict__ dd = gpu(it.d + sd.offset);
  const gmem<const dv2> *__restrict__ tw = gpu((const dv2 *)sd.tw);
  const gmem<const dv2> *__restrict__ ptw = gpu((const dv2 *)sd.ptw);
  const int len = uni((int)sd.length);
  const double inv_m = 1.0 / (double)(4 * h);
  auto wm = [&](int r) {
    const dv2 v = tw[r];
    return make_double2(v.x, -v.y);
  };
  auto stage = [&](int s, bool odd) {
    t = opaque_tid();
    for (int i0 = 0; i0 < NI; i0 += RL_CH) {
      double rv[RL_CH][2];
#pragma unroll
      for (int c = 0; c < RL_CH; ++c)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int jj = 2 * P * (t + RL_THREADS * (i0 + c)) + 2 * s + u;
          rv[c][u] = jj < len ? dd[jj] - hrow[jj] : 0.0;
        }
#pragma unroll
      for (int c = 0; c < RL_CH; ++c) {
        const int n = t + RL_THREADS * (i0 + c);
        const double2 z = make_double2(rv[c][0], rv[c][1]);
        X[lpad(n)] = odd ? cmul(z, wm(2 * P * n + 2 * s)) : z;
      }
    }
    __syncthreads();
  };
  auto mult = [&](int r) { return from_dv2(M[r]); };
  double ss = 0.0;
  // even part parked in this workgroup's scratch (the same thread reads it back)
  auto emit = [&](int s, bool odd) {
    t = opaque_tid();
    for (int i = 0; i < NI; ++i) {
      const int n = t + RL_THREADS * i, j0 = 2 * P * n + 2 * s;
      if (j0 >= len) continue;
      if (!odd) {
        const double2 g = X[lpad(n)];
        tes[j0] = g.x;
        if (j0 + 1 < len) tes[j0 + 1] = -g.y;
        continue;
      }
      const double2 gz = conj2(cmul(wm(j0), X[lpad(n)]));
      const double c0 = (tes[j0] + gz.x) * inv_m;
      ss += c0 * c0;
      if (j0 + 1 < len) {
        const double c1 = (tes[j0 + 1] + gz.y) * inv_m;
        ss += c1 * c1;
      }
    }
  };
  if constexpr (P == 2)
    rl_split_parts<LH>(X, tw, ptw, stage, mult, emit);
  else
    rl_quad_parts<LH>(X, S, tw, ptw, stage, mult, emit);
  return ss;
}

template <int LH>
__device__ __forceinline__ void gs_segment(const GsItem &it, const GsSeg &sd, int64_t b, double2 *X,
                                           gmem<double> *__restrict__ tes, double &qacc) {
  qacc += gs_pair<LH>(it, sd, b, gp((const dv2 *)sd.M1), gp((const dv2 *)sd.M2), X, tes) *
          sd.inv_x0;
}

// Per-workgroup scratch of `stride` doubles: the parked even part, then (qoff >= 0) the
// quarters of transforms split in four.
__global__ __launch_bounds__(RL_THREADS) void k_gs(const GsItem *__restrict__ items,
                                                   const int2 *__restrict__ work, int64_t n_work,
                                                   double *__restrict__ scratch, int64_t stride,
                                                   int64_t qoff) {
  extern __shared__ double2 rl_smem[];
  double2 *X = rl_smem;
  double *red = (double *)(rl_smem + RL_XN);
  gmem<double> *tes = gpu(scratch + (int64_t)blockIdx.x * stride);
  gmem<dv2> *S = qoff >= 0 ? (gmem<dv2> *)(tes + qoff) : nullptr;
  for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
    const int2 wk = work[wi];
    if (wk.x < 0) continue;  // padding of the work list
    const GsItem &it = items[wk.x];
    const int64_t b = wk.y;
    double qp = 0.0;
    bool bad = false;
    for (int sg = 0; sg < it.n_segs; ++sg) {
      const GsSeg sd = it.segs[sg];
      switch (sd.log2m - 2) {
#define TDA_GS(LH) \
  case LH: gs_segment<LH>(it, sd, b, X, tes, qp); break;
        TDA_GS(2) TDA_GS(3) TDA_GS(4) TDA_GS(5) TDA_GS(6) TDA_GS(7) TDA_GS(8) TDA_GS(9)
        TDA_GS(10) TDA_GS(11) TDA_GS(12) TDA_GS(13)
#undef TDA_GS
        case RL_LHMAX + 1: {
          const double s1 =
              gs_sumsq_split<RL_LHMAX + 1, 2>(it, sd, b, gp((const dv2 *)sd.M1), X, nullptr, tes);
          const double s2 =
              gs_sumsq_split<RL_LHMAX + 1, 2>(it, sd, b, gp((const dv2 *)sd.M2), X, nullptr, tes);
          qp += (s1 - s2) * sd.inv_x0;
          break;
        }
        case RL_LHMAX + 2: {
          if (!S) {
            bad = true;
            break;
          }
          const double s1 =
              gs_sumsq_split<RL_LHMAX + 2, 4>(it, sd, b, gp((const dv2 *)sd.M1), X, S, tes);
          const double s2 =
              gs_sumsq_split<RL_LHMAX + 2, 4>(it, sd, b, gp((const dv2 *)sd.M2), X, S, tes);
          qp += (s1 - s2) * sd.inv_x0;
          break;
        }
        default: bad = true;
      }
    }
    double q[1] = {bad ? __builtin_nan("") : qp};
    block_sum0(q, red);
    if (threadIdx.x == 0) it.out[b] = -0.5 * q[0] + it.cterm;
  }
}

hipError_t launch_gs(const GsItem *items, const int2 *work, int64_t n_work, double *scratch,
                     int64_t scratch_stride, int64_t qoff, int32_t n_wg, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>(n_work, n_wg);
  hipLaunchKernelGGL(k_gs, dim3((unsigned)g), dim3(RL_THREADS), RL_LDS_BYTES, s, items, work, n_work,
                     scratch, scratch_stride, qoff);
  return hipGetLastError();
}

void register_mixed_attributes() {
  hipFuncSetAttribute((const void *)k_trmm_fwd<5>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)PL<5>::lds_bytes());
  hipFuncSetAttribute((const void *)k_trmm_bwd<5>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)PL<5>::lds_bytes());
  hipFuncSetAttribute((const void *)k_corr<5>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)PL<5>::lds_bytes());
  hipFuncSetAttribute((const void *)k_refine_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)RL_LDS_BYTES);
  hipFuncSetAttribute((const void *)k_gs, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)RL_LDS_BYTES);
  hipFuncSetAttribute((const void *)k_levinson<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)(RL_MAX_LEV * sizeof(double)));
}

}  // namespace tda
