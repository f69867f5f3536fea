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

// round-to-nearest-even FP32 -> BF16 bits (NaN kept NaN)
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
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

__device__ __forceinline__ bf8 load_frag(const uint16_t *p) {
  return *reinterpret_cast<const bf8 *>(p);
}

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
// the whitened data vector is computed once and cached).
__global__ void k_dbar(const double *__restrict__ w64, const int64_t *__restrict__ off,
                       const int32_t *__restrict__ rb, const int32_t *__restrict__ blk_first,
                       const int32_t *__restrict__ idx, const double *__restrict__ d,
                       double *__restrict__ dbar) {
  const int i = blockIdx.x;
  const int64_t r = (int64_t)i * TB + threadIdx.x;
  const int64_t c_beg = (int64_t)blk_first[i] * TB;
  double acc = 0.0;
  for (int64_t c = c_beg; c <= r; ++c) {
    const int32_t p = idx[c];
    if (p < 0) continue;
    acc += w64_at(w64, off, rb, r, c) * d[p];
  }
  dbar[r] = acc;
}

__global__ void k_yd(const double *__restrict__ w64, const int64_t *__restrict__ off,
                     const int32_t *__restrict__ rb, const int32_t *__restrict__ blk_last,
                     const double *__restrict__ dbar, double *__restrict__ yd) {
  __shared__ double part[8][32];
  const int ct = blockIdx.x;
  const int cc = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int64_t c = (int64_t)ct * 32 + cc;
  const int64_t r_end = (int64_t)(blk_last[c / TB] + 1) * TB;
  double acc = 0.0;
  for (int64_t r = rb[ct] + g; r < r_end; r += 8) acc += w64_at(w64, off, rb, r, c) * dbar[r];
  part[g][cc] = acc;
  __syncthreads();
  if (g == 0) {
    double s = 0.0;
    for (int k = 0; k < 8; ++k) s += part[k][cc];
    yd[c] = s;
  }
}

__global__ void k_qdd_and_scatter(const double *__restrict__ dbar, const double *__restrict__ yd,
                                  const int32_t *__restrict__ idx, int32_t n_pad, int64_t N,
                                  double *__restrict__ yd_pos, double *__restrict__ qdd) {
  __shared__ double part[256];
  for (int64_t j = threadIdx.x; j < N; j += 256) yd_pos[j] = 0.0;
  __syncthreads();
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n_pad; r += 256) {
    s += dbar[r] * dbar[r];
    const int32_t p = idx[r];
    if (p >= 0) yd_pos[p] = yd[r];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 256; ++k) t += part[k];
    qdd[0] = t;
  }
}

hipError_t launch_data_whiten(const double *w64, const int64_t *w64_off, const int32_t *w64_rb,
                              const int32_t *blk_first, const int32_t *blk_last, const int32_t *idx,
                              int32_t n_pad, int64_t N, const double *d, double *dbar, double *yd,
                              double *yd_pos, double *qdd, hipStream_t s) {
  hipLaunchKernelGGL(k_dbar, dim3((unsigned)(n_pad / TB)), dim3(TB), 0, s, w64, w64_off, w64_rb,
                     blk_first, idx, d, dbar);
  hipLaunchKernelGGL(k_yd, dim3((unsigned)(n_pad / 32)), dim3(256), 0, s, w64, w64_off, w64_rb,
                     blk_last, dbar, yd);
  hipLaunchKernelGGL(k_qdd_and_scatter, dim3(1), dim3(256), 0, s, dbar, yd, idx, n_pad, N, yd_pos,
                     qdd);
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

hipError_t launch_lambda(const double *acf, int64_t length, int64_t m, double *tw, double *lam,
                         hipStream_t s) {
  const unsigned g = (unsigned)((m + 255) / 256);
  hipLaunchKernelGGL(k_twiddles, dim3(g), dim3(256), 0, s, m, tw);
  hipLaunchKernelGGL(k_lambda, dim3(g), dim3(256), 0, s, acf, length, m, tw, lam);
  return hipGetLastError();
}

// ---------------------------------------------------------------- template split
// F(Hs): rows = templates (padded to Bp), K = padded sample rows; Hs[b][p] = h_b[idx[p]].
__global__ void k_split_h(const MixItem *__restrict__ items, int32_t item_id, int64_t chunks) {
  const int64_t chunk = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (chunk >= chunks) return;
  const MixItem &it = items[item_id];
  const int64_t nks = it.n_pad / 16;
  const int lane = (int)(chunk & 63);
  const int64_t ks = (chunk >> 6) % nks;
  const int64_t tt = (chunk >> 6) / nks;
  const int64_t b = 32 * tt + (lane & 31);
  const int64_t p0 = 16 * ks + 8 * (lane >> 5);
  uint16_t hi[8], lo[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    double v = 0.0;
    const int32_t p = it.idx[p0 + e];
    if (b < it.B && p >= 0) v = template_row(it, b)[p];
    split2(v, hi[e], lo[e]);
  }
  uint4 vh, vl;
  vh.x = hi[0] | ((uint32_t)hi[1] << 16); vh.y = hi[2] | ((uint32_t)hi[3] << 16);
  vh.z = hi[4] | ((uint32_t)hi[5] << 16); vh.w = hi[6] | ((uint32_t)hi[7] << 16);
  vl.x = lo[0] | ((uint32_t)lo[1] << 16); vl.y = lo[2] | ((uint32_t)lo[3] << 16);
  vl.z = lo[4] | ((uint32_t)lo[5] << 16); vl.w = lo[6] | ((uint32_t)lo[7] << 16);
  *reinterpret_cast<uint4 *>(it.hs_hi + chunk * 8) = vh;
  *reinterpret_cast<uint4 *>(it.hs_lo + chunk * 8) = vl;
}

hipError_t launch_split_h(const MixItem *items, int32_t item_id, int64_t Bp, int64_t n_pad,
                          hipStream_t s) {
  const int64_t chunks = (Bp / 32) * (n_pad / 16) * 64;
  hipLaunchKernelGGL(k_split_h, dim3((unsigned)((chunks + 255) / 256)), dim3(256), 0, s, items,
                     item_id, chunks);
  return hipGetLastError();
}

// ---------------------------------------------------------------- BF16x3 products
// Work entry: (item, block, template group of MT = 128, unused); block < 0 = idle.
// Workgroup tile 256 rows x 128 templates; wave w: rows 128 (w/2) .. +128 (4 tiles),
// templates 64 (w%2) .. +64 (2 tiles).  Each product accumulates hi*hi + hi*lo + lo*hi.

__global__ __launch_bounds__(256, 2) void k_trmm_fwd(const MixItem *__restrict__ items,
                                                     const int4 *__restrict__ work) {
  const int4 wk = work[blockIdx.x];
  if (wk.y < 0) return;
  const MixItem &it = items[wk.x];
  const int i = wk.y, tg = wk.z;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int bf = it.blk_first[i];
  const int64_t nks = (int64_t)(i + 1 - bf) * (TB / 16);
  const int64_t nks_all = it.n_pad / 16;
  const int64_t ks0 = (int64_t)bf * (TB / 16);
  const uint16_t *Ah = it.wa_hi + it.wa_off[i] + (int64_t)(4 * (w >> 1)) * 512 + lane * 8;
  const uint16_t *Al = it.wa_lo + it.wa_off[i] + (int64_t)(4 * (w >> 1)) * 512 + lane * 8;
  const int64_t T0 = (int64_t)tg * 4 + 2 * (w & 1);  // first template tile of this wave
  const uint16_t *Bh = it.hs_hi + ((T0 * nks_all + ks0) * 64 + lane) * 8;
  const uint16_t *Bl = it.hs_lo + ((T0 * nks_all + ks0) * 64 + lane) * 8;
  const int64_t bstride = nks_all * 512;  // next template tile
  f16v acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f16v{};
  for (int64_t ks = 0; ks < nks; ++ks) {
    bf8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ah[a] = load_frag(Ah + (ks * 8 + a) * 512);
      al[a] = load_frag(Al + (ks * 8 + a) * 512);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      bh[b] = load_frag(Bh + b * bstride + ks * 512);
      bl[b] = load_frag(Bl + b * bstride + ks * 512);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        acc[a][b] = mfma_bf16(ah[a], bh[b], acc[a][b]);
        acc[a][b] = mfma_bf16(ah[a], bl[b], acc[a][b]);
        acc[a][b] = mfma_bf16(al[a], bh[b], acc[a][b]);
      }
  }
  // w0 in F(w0^T): element (template b, row p) -> tile b/32, kstep p/16,
  // lane b%32 + 32 ((p%16)/8), position p%8.
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t rt_row = (int64_t)i * TB + 128 * (w >> 1) + 32 * a;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t T = T0 + b;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t base = rt_row + 8 * g;         // multiple of 8
        const int64_t ks = base >> 4;
        const int lp = (lane & 31) + 32 * (g & 1);
        const int64_t dst = ((T * nks_all + ks) * 64 + lp) * 8 + 4 * (lane >> 5);
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

// y0^T = w0^T W over column block j: K = rows [j TB, (last_j + 1) TB).
// Workgroup tile 128 templates x 256 samples; wave w: templates 64 (w/2) (2 tiles),
// samples 128 (w%2) (4 tiles).
__global__ __launch_bounds__(256, 2) void k_trmm_bwd(const MixItem *__restrict__ items,
                                                     const int4 *__restrict__ work) {
  const int4 wk = work[blockIdx.x];
  if (wk.y < 0) return;
  const MixItem &it = items[wk.x];
  const int j = wk.y, tg = wk.z;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int last = it.blk_last[j];
  const int64_t nks = (int64_t)(last + 1 - j) * (TB / 16);
  const int64_t nks_all = it.n_pad / 16;
  const int64_t ks0 = (int64_t)j * (TB / 16);
  const int64_t T0 = (int64_t)tg * 4 + 2 * (w >> 1);
  const uint16_t *Ah = it.w0_hi + ((T0 * nks_all + ks0) * 64 + lane) * 8;
  const uint16_t *Al = it.w0_lo + ((T0 * nks_all + ks0) * 64 + lane) * 8;
  const int64_t astride = nks_all * 512;
  const int st0 = 4 * (w & 1);
  const uint16_t *Bh = it.wb_hi + it.wb_off[j] + (int64_t)st0 * 512 + lane * 8;
  const uint16_t *Bl = it.wb_lo + it.wb_off[j] + (int64_t)st0 * 512 + lane * 8;
  f16v acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f16v{};
  for (int64_t ks = 0; ks < nks; ++ks) {
    bf8 ah[2], al[2], bh[4], bl[4];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      ah[a] = load_frag(Ah + a * astride + ks * 512);
      al[a] = load_frag(Al + a * astride + ks * 512);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      bh[b] = load_frag(Bh + (ks * 8 + b) * 512);
      bl[b] = load_frag(Bl + (ks * 8 + b) * 512);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[a][b] = mfma_bf16(ah[a], bh[b], acc[a][b]);
        acc[a][b] = mfma_bf16(ah[a], bl[b], acc[a][b]);
        acc[a][b] = mfma_bf16(al[a], bh[b], acc[a][b]);
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int64_t trow0 = 32 * (T0 + a);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t col = (int64_t)j * TB + 32 * (st0 + b) + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t trow = trow0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        it.y0[trow * it.n_pad + col] = acc[a][b][r];
      }
    }
  }
}

hipError_t launch_trmm_fwd(const MixItem *items, const int4 *work, int64_t n_work, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trmm_fwd, dim3((unsigned)n_work), dim3(256), 0, s, items, work);
  return hipGetLastError();
}

hipError_t launch_trmm_bwd(const MixItem *items, const int4 *work, int64_t n_work, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trmm_bwd, dim3((unsigned)n_work), dim3(256), 0, s, items, work);
  return hipGetLastError();
}

// ---------------------------------------------------------------- FP64 refinement
// Per template and segment: x = y0 scattered to the segment's sample positions (0 at
// excluded samples and beyond the segment), X = DFT_m(x), and
//   y0^T C y0 = (1/m) sum_k lambda_k |X_k|^2     (circulant embedding, eq:toeplitz_fft)
// The refined quadratic form s_hat = 2 h^T y0 - y0^T C y0 <= h^T C^-1 h with error
// (y* - y0)^T C (y* - y0), and q = q_dd - 2 y_d^T h + s_hat (all FP64).
// The length-m DFT is two passes of radix-2 FFTs of lengths n1, n2 (m = n1 n2) in LDS
// with the intermediate in the workgroup's global scratch.

constexpr int FFT_LDS = 4096;  // complex doubles staged in LDS (64 KiB)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// forward radix-2 DIT on `cols` columns of length P stored bit-reversed in X[c*P + .]
__device__ void fft_cols(double2 *X, int cols, int P, int logP, int64_t m, const double *tw) {
  const int64_t tstep = m / P;
  for (int s = 1; s <= logP; ++s) {
    const int half = 1 << (s - 1);
    const int total = cols * (P >> 1);
    for (int u = threadIdx.x; u < total; u += blockDim.x) {
      const int c = u / (P >> 1), v = u % (P >> 1);
      const int grp = v >> (s - 1), o = v & (half - 1);
      const int i0 = c * P + (grp << s) + o, i1 = i0 + half;
      const int64_t r = (int64_t)o * (P >> s) * tstep;  // twiddle exponent in units of 1/m
      const double2 wv = make_double2(tw[2 * r], -tw[2 * r + 1]);
      const double2 a = X[i0], b = cmul(X[i1], wv);
      X[i0] = make_double2(a.x + b.x, a.y + b.y);
      X[i1] = make_double2(a.x - b.x, a.y - b.y);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

__device__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)blockDim.x; ++k) s += red[k];
  __syncthreads();
  return s;  // valid on thread 0
}

__global__ __launch_bounds__(256) void k_refine(const RefItem *__restrict__ items,
                                                const int2 *__restrict__ work, int64_t n_work,
                                                double2 *__restrict__ scratch_all,
                                                int64_t scratch_per_wg) {
  __shared__ double2 X[FFT_LDS];
  __shared__ double red[256];
  double2 *S = scratch_all + (int64_t)blockIdx.x * scratch_per_wg;
  for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
    const int2 wk = work[wi];
    const RefItem &it = items[wk.x];
    const int64_t b = wk.y;
    const float *y = it.y0 + b * it.n_pad;
    const double *h = template_row(it, b);
    double hy = 0.0, ydh = 0.0, quad_total = 0.0;
    for (int sg = 0; sg < it.n_segs; ++sg) {
      const SegDev sd = it.segs[sg];
      const int log2m = sd.log2m;
      const int l1 = (log2m + 1) / 2, l2 = log2m / 2;
      const int n1 = 1 << l1, n2 = 1 << l2;
      const int64_t m = sd.m;
      // pass 1: columns j2 (stride n2), length n1
      const int cb1 = FFT_LDS / n1;
      for (int j2b = 0; j2b < n2; j2b += cb1) {
        const int cols = min(cb1, n2 - j2b);
        for (int u = threadIdx.x; u < cols * n1; u += blockDim.x) {
          const int c = u % cols, j1 = u / cols;
          const int64_t jpos = (int64_t)n2 * j1 + j2b + c;
          double xv = 0.0;
          if (jpos < sd.length) {
            const int32_t p = it.pos2row[sd.offset + jpos];
            if (p >= 0) {
              xv = (double)y[p];
              const double hv = h[sd.offset + jpos];
              hy += hv * xv;
              ydh += hv * it.yd_pos[sd.offset + jpos];
            }
          }
          X[c * n1 + bitrev(j1, l1)] = make_double2(xv, 0.0);
        }
        __syncthreads();
        fft_cols(X, cols, n1, l1, m, sd.tw);
        for (int u = threadIdx.x; u < cols * n1; u += blockDim.x) {
          const int c = u % cols, k1 = u / cols;
          const int64_t j2 = j2b + c;
          const int64_t r = (j2 * (int64_t)k1) & (m - 1);
          const double2 wv = make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]);
          S[(int64_t)k1 * n2 + j2] = cmul(X[c * n1 + k1], wv);
        }
        __threadfence_block();
        __syncthreads();
      }
      // pass 2: rows k1, length n2 over j2
      const int cb2 = FFT_LDS / n2;
      double quad = 0.0;
      for (int k1b = 0; k1b < n1; k1b += cb2) {
        const int rows = min(cb2, n1 - k1b);
        for (int u = threadIdx.x; u < rows * n2; u += blockDim.x) {
          const int c = u / n2, j2 = u % n2;
          X[c * n2 + bitrev(j2, l2)] = S[(int64_t)(k1b + c) * n2 + j2];
        }
        __syncthreads();
        fft_cols(X, rows, n2, l2, m, sd.tw);
        for (int u = threadIdx.x; u < rows * n2; u += blockDim.x) {
          const int c = u / n2, k2 = u % n2;
          const double2 v = X[c * n2 + k2];
          quad += sd.lam[(int64_t)(k1b + c) + (int64_t)n1 * k2] * (v.x * v.x + v.y * v.y);
        }
        __syncthreads();
      }
      quad_total += quad / (double)m;
    }
    const double s_hy = block_sum(hy, red);
    const double s_ydh = block_sum(ydh, red);
    const double s_quad = block_sum(quad_total, red);
    if (threadIdx.x == 0) {
      const double shat = 2.0 * s_hy - s_quad;
      const double q = it.qdd[0] - 2.0 * s_ydh + shat;
      it.out[b] = -0.5 * q + it.cterm;
    }
  }
}

hipError_t launch_refine(const RefItem *items, const int2 *work, int64_t n_work, double *scratch,
                         int64_t scratch_per_wg, int32_t n_wg, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine, dim3((unsigned)n_wg), dim3(256), 0, s, items, work, n_work,
                     (double2 *)scratch, scratch_per_wg / 2);
  return hipGetLastError();
}

}  // namespace tda
