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
// grid (chunks of the largest item, items); each item has (Bp/32) (n_pad/16) 64 chunks
__global__ void k_split_h(const MixItem *__restrict__ items, int from_e) {
  const MixItem &it = items[blockIdx.y];
  const int64_t nks = it.n_pad / 16;
  const int64_t chunks = (int64_t)(it.Bp / 32) * nks * 64;
  const int64_t chunk = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (chunk >= chunks || it.B == 0) return;
  const int lane = (int)(chunk & 63);
  const int64_t ks = (chunk >> 6) % nks;
  const int64_t tt = (chunk >> 6) / nks;
  const int64_t b = 32 * tt + (lane & 31);
  const int64_t p0 = 16 * ks + 8 * (lane >> 5);
  uint16_t hi[8], lo[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    double v = 0.0;
    if (from_e) {
      if (b < it.B) v = it.e64[b * it.n_pad + p0 + e];
    } else {
      const int32_t p = it.idx[p0 + e];
      if (b < it.B && p >= 0) v = template_row(it, b)[p];
    }
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

hipError_t launch_split_h(const MixItem *items, int32_t n_items, int64_t max_chunks, int from_e,
                          hipStream_t s) {
  if (n_items <= 0 || max_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_h, dim3((unsigned)((max_chunks + 255) / 256), (unsigned)n_items),
                     dim3(256), 0, s, items, from_e);
  return hipGetLastError();
}

// ---------------------------------------------------------------- BF16x3 products
// A workgroup (4 waves) computes a 256 x 128 tile of D = A B over K = 16 nks; A and B are
// given as fragment arrays: A tile t (32 rows) at k-step ks is at A + t s_tile + ks s_ks.
// Wave w owns A tiles 4 (w/2) .. +4 and B tiles 2 (w%2) .. +2 (a 128 x 64 sub-tile).
// Fragments go straight from HBM/L2 into registers, one k-step ahead of the matrix
// cores.  Every product is hi*hi + hi*lo + lo*hi with FP32 accumulation.
struct FragSrc {
  const uint16_t *hi, *lo;
  int64_t s_tile, s_ks;  // element strides between tiles and between k-steps
};

constexpr int FRAG = 512;  // bf16 elements per fragment (64 lanes x 8)

struct Step {
  bf8 ah[4], al[4], bh[2], bl[2];
};

// NPROD = 3: hi*hi + hi*lo + lo*hi; NPROD = 1: hi*hi only (lo parts not loaded)
template <int NPROD>
__device__ __forceinline__ void load_step(const FragSrc &A, const FragSrc &B, int ta, int tb,
                                          int64_t ks, int lane, Step &st) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t off = (int64_t)(ta + a) * A.s_tile + ks * A.s_ks + lane * 8;
    st.ah[a] = load_frag(A.hi + off);
    if (NPROD == 3) st.al[a] = load_frag(A.lo + off);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int64_t off = (int64_t)(tb + b) * B.s_tile + ks * B.s_ks + lane * 8;
    st.bh[b] = load_frag(B.hi + off);
    if (NPROD == 3) st.bl[b] = load_frag(B.lo + off);
  }
}

template <int NPROD>
__device__ __forceinline__ void mma_step(const Step &st, f16v (&acc)[4][2]) {
  // separate passes so consecutive matrix-core ops use independent accumulators
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = mfma_bf16(st.ah[a], st.bh[b], acc[a][b]);
  if (NPROD == 3) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma_bf16(st.ah[a], st.bl[b], acc[a][b]);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma_bf16(st.al[a], st.bh[b], acc[a][b]);
  }
}

template <int NPROD = 3>
__device__ __forceinline__ void gemm3(const FragSrc &A, const FragSrc &B, int64_t nks,
                                      f16v (&acc)[4][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ta = 4 * (w >> 1), tb = 2 * (w & 1);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f16v{};
  Step s0, s1;
  if (nks > 0) load_step<NPROD>(A, B, ta, tb, 0, lane, s0);
  int64_t ks = 0;
  for (; ks + 1 < nks; ks += 2) {
    load_step<NPROD>(A, B, ta, tb, ks + 1, lane, s1);
    mma_step<NPROD>(s0, acc);
    if (ks + 2 < nks) load_step<NPROD>(A, B, ta, tb, ks + 2, lane, s0);
    mma_step<NPROD>(s1, acc);
  }
  if (ks < nks) mma_step<NPROD>(s0, acc);
}

// w0 = W h: rows of row block i, templates of group tg (128); w0 written as F(w0^T).
template <int OCC>
__global__ __launch_bounds__(256, OCC) void k_trmm_fwd(const MixItem *__restrict__ items,
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
  const int64_t T0 = (int64_t)tg * 4;
  const FragSrc A{it.wa_hi + it.wa_off[i], it.wa_lo + it.wa_off[i], FRAG, 8 * FRAG};
  const FragSrc B{it.hs_hi + (T0 * nks_all + ks0) * FRAG, it.hs_lo + (T0 * nks_all + ks0) * FRAG,
                  nks_all * FRAG, FRAG};
  f16v acc[4][2];
  gemm3(A, B, nks, acc);
  // element (template b, row p) of F(w0^T): tile b/32, kstep p/16, lane b%32 + 32((p%16)/8), pos p%8
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t rt_row = (int64_t)i * TB + 32 * (4 * (w >> 1) + a);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t T = T0 + 2 * (w & 1) + b;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t base = rt_row + 8 * g;
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

// y0^T = w0^T W over column block j (K = rows [j TB, (last_j + 1) TB)): A = F(w0^T)
// (256 templates of group tg), B = F(W^T) restricted to half `hf` (128 samples) of block j.
template <int OCC>
__global__ __launch_bounds__(256, OCC) void k_trmm_bwd(const MixItem *__restrict__ items,
                                                     const int4 *__restrict__ work) {
  const int4 wk = work[blockIdx.x];
  if (wk.y < 0) return;
  const MixItem &it = items[wk.x];
  const int j = wk.y, tg = wk.z, hf = wk.w;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int last = it.blk_last[j];
  const int64_t nks = (int64_t)(last + 1 - j) * (TB / 16);
  const int64_t nks_all = it.n_pad / 16;
  const int64_t ks0 = (int64_t)j * (TB / 16);
  const int64_t T0 = (int64_t)tg * 8;
  const FragSrc A{it.w0_hi + (T0 * nks_all + ks0) * FRAG, it.w0_lo + (T0 * nks_all + ks0) * FRAG,
                  nks_all * FRAG, FRAG};
  const FragSrc B{it.wb_hi + it.wb_off[j] + (int64_t)hf * 4 * FRAG,
                  it.wb_lo + it.wb_off[j] + (int64_t)hf * 4 * FRAG, FRAG, 8 * FRAG};
  f16v acc[4][2];
  gemm3(A, B, nks, acc);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t trow0 = 32 * (T0 + 4 * (w >> 1) + a);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t col = (int64_t)j * TB + 32 * (4 * hf + 2 * (w & 1) + b) + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t trow = trow0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        it.y0[trow * it.n_pad + col] = acc[a][b][r];
      }
    }
  }
}

// Correction c_b = ||W e_b||^2: same product as the forward one with the split residual
// (in the template buffers) as B; the epilogue writes, per template, the sum of squares
// over the 256 rows of block i to corr_part[i][b] (fixed order, no atomics).  The
// correction only has to be accurate relative to itself (it is already second order in
// the product error); CORR_PROD selects 3 (hi*hi + hi*lo + lo*hi) or 1 (hi*hi) products.
constexpr int CORR_PROD = 3;
template <int OCC>
__global__ __launch_bounds__(256, OCC) void k_corr(const MixItem *__restrict__ items,
                                                 const int4 *__restrict__ work) {
  __shared__ double red[2][128];
  const int4 wk = work[blockIdx.x];
  if (wk.y < 0) return;
  const MixItem &it = items[wk.x];
  const int i = wk.y, tg = wk.z;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int bf = it.blk_first[i];
  const int64_t nks = (int64_t)(i + 1 - bf) * (TB / 16);
  const int64_t nks_all = it.n_pad / 16;
  const int64_t ks0 = (int64_t)bf * (TB / 16);
  const int64_t T0 = (int64_t)tg * 4;
  const FragSrc A{it.wa_hi + it.wa_off[i], it.wa_lo + it.wa_off[i], FRAG, 8 * FRAG};
  const FragSrc B{it.hs_hi + (T0 * nks_all + ks0) * FRAG, it.hs_lo + (T0 * nks_all + ks0) * FRAG,
                  nks_all * FRAG, FRAG};
  f16v acc[4][2];
  gemm3<CORR_PROD>(A, B, nks, acc);
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    double ss = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) ss += (double)acc[a][b][r] * (double)acc[a][b][r];
    ss += __shfl_xor(ss, 32);  // lanes l and l+32 hold other rows of the same column
    const int col = 32 * (2 * (w & 1) + b) + (lane & 31);
    if (lane < 32) red[w >> 1][col] = ss;
  }
  __syncthreads();
  if (threadIdx.x < 128) {
    const int col = threadIdx.x;
    it.corr_part[(int64_t)i * it.Bp + T0 * 32 + col] = red[0][col] + red[1][col];
  }
}

// out[b] = -1/2 (qpart[b] + sum_i corr_part[i][b]) + cterm; entries (item, b)
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
}

// variant: waves per SIMD the kernel is compiled for (1: no register spills, operands
// and accumulators fully resident; 2: two workgroups per CU for more latency hiding)
#define TDA_LAUNCH_VARIANT(K)                                                                 \
  if (n_work <= 0) return hipSuccess;                                                        \
  if (variant == 2)                                                                          \
    hipLaunchKernelGGL(K<2>, dim3((unsigned)n_work), dim3(256), 0, s, items, work);           \
  else                                                                                       \
    hipLaunchKernelGGL(K<1>, dim3((unsigned)n_work), dim3(256), 0, s, items, work);           \
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

void register_mixed_attributes() {}

// ---------------------------------------------------------------- FP64 refinement
// Per template pair (a, b) and segment: x = y0 scattered to the segment's sample
// positions (0 at excluded samples and beyond the segment), z = x_a + i x_b, and
//   C x = first `length` entries of IDFT_m(lambda . DFT_m(z))   (real part: a, imag: b)
// because C is the leading block of the circulant of length m >= 2 length whose first
// column embeds the ACF (eq:toeplitz_fft; lambda real and even, so the two real
// sequences separate in the real and imaginary parts).  With e = h - C y0 (FP64):
//   s_hat = 2 h^T y0 - y0^T C y0 <= h^T C^-1 h, error (y* - y0)^T C (y* - y0) = e^T C^-1 e,
// and the correction kernel adds ||W e||^2, leaving an error of third order.
//   qpart = q_dd - 2 y_d^T h + s_hat        (FP64), e written for the correction.
// The length-m DFTs are four-step (m = n1 n2): n1-point DFTs down the columns of x seen
// as n1 x n2 row-major, twiddle, n2-point DFTs along rows; the inverse runs the same
// steps backwards.  Small DFTs are radix-4/2 Stockham sequences in LDS; the intermediate
// lives in the workgroup's global scratch.

constexpr int FFT_BUF = 2048;  // complex doubles per LDS buffer (two buffers, ping-pong)
constexpr int FFT_THREADS = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

// Forward DFT of `cols` sequences of length P = 2^logP at X[c*P + j] (natural order in and
// out); returns the buffer (X or Y) holding the result.  twP[k] = exp(-2 pi i k / P).
__device__ double2 *dft_lds(double2 *X, double2 *Y, int cols, int logP, const double2 *twP) {
  const int P = 1 << logP;
  int Ns = 1;
  double2 *src = X, *dst = Y;
  int left = logP;
  while (left > 0) {
    if (left >= 2) {  // radix-4 stage
      const int quarter = P >> 2;
      const int total = cols * quarter;
      for (int u = threadIdx.x; u < total; u += blockDim.x) {
        const int c = u >> (logP - 2), j = u & (quarter - 1);
        const double2 *in = src + c * P;
        double2 *out = dst + c * P;
        const int k = j & (Ns - 1);
        const int tstride = P / (Ns * 4);
        double2 v0 = in[j], v1 = in[j + quarter], v2 = in[j + 2 * quarter], v3 = in[j + 3 * quarter];
        if (Ns > 1) {
          v1 = cmul(v1, twP[(k * tstride) & (P - 1)]);
          v2 = cmul(v2, twP[(2 * k * tstride) & (P - 1)]);
          v3 = cmul(v3, twP[(3 * k * tstride) & (P - 1)]);
        }
        const double2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3);
        const double2 d = csub(v1, v3);
        const double2 a3 = make_double2(d.y, -d.x);  // -i (v1 - v3)
        const int base = (j / Ns) * Ns * 4 + k;
        out[base] = cadd(a0, a2);
        out[base + Ns] = cadd(a1, a3);
        out[base + 2 * Ns] = csub(a0, a2);
        out[base + 3 * Ns] = csub(a1, a3);
      }
      Ns *= 4;
      left -= 2;
    } else {  // radix-2 stage
      const int half = P >> 1;
      const int total = cols * half;
      for (int u = threadIdx.x; u < total; u += blockDim.x) {
        const int c = u >> (logP - 1), j = u & (half - 1);
        const double2 *in = src + c * P;
        double2 *out = dst + c * P;
        const int k = j & (Ns - 1);
        double2 v0 = in[j], v1 = in[j + half];
        if (Ns > 1) v1 = cmul(v1, twP[(k * (P / (Ns * 2))) & (P - 1)]);
        const int base = (j / Ns) * Ns * 2 + k;
        out[base] = cadd(v0, v1);
        out[base + Ns] = csub(v0, v1);
      }
      Ns *= 2;
      left -= 1;
    }
    __syncthreads();
    double2 *t = src;
    src = dst;
    dst = t;
  }
  return src;
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

// Work entry: (item, template a, template b or -1, 0).
__global__ __launch_bounds__(FFT_THREADS) void k_refine(const RefItem *__restrict__ items,
                                                        const int4 *__restrict__ work,
                                                        int64_t n_work,
                                                        double2 *__restrict__ scratch_all,
                                                        int64_t scratch_per_wg) {
  __shared__ double2 buf[2][FFT_BUF];
  __shared__ double2 tw1[512], tw2[512];
  __shared__ double red[FFT_THREADS];
  double2 *S = scratch_all + (int64_t)blockIdx.x * scratch_per_wg;
  for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
    const int4 wk = work[wi];
    const RefItem &it = items[wk.x];
    const int64_t ba = wk.y, bb = wk.z;
    const bool two = bb >= 0;
    const float *ya = it.y0 + ba * it.n_pad;
    const float *yb = it.y0 + (two ? bb : ba) * it.n_pad;
    const double *ha = template_row(it, ba);
    const double *hb = template_row(it, two ? bb : ba);
    double *ea = it.e64 + ba * it.n_pad;
    double *eb = two ? it.e64 + bb * it.n_pad : nullptr;
    double hy_a = 0, hy_b = 0, ydh_a = 0, ydh_b = 0, yc_a = 0, yc_b = 0;
    // a non-finite y0 entry must not reach the partner through the shared DFT: it is
    // replaced by 0 there and the template's result is set to NaN at the end
    double bad_a = 0, bad_b = 0;
    for (int sg = 0; sg < it.n_segs; ++sg) {
      const SegDev sd = it.segs[sg];
      const int log2m = sd.log2m;
      const int l1 = (log2m + 1) / 2, l2 = log2m / 2;
      const int n1 = 1 << l1, n2 = 1 << l2;
      const int64_t m = sd.m;
      const double inv_m = 1.0 / (double)m;
      for (int k = threadIdx.x; k < n1; k += blockDim.x) {
        const int64_t r = (int64_t)k * (m / n1);
        tw1[k] = make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]);
      }
      for (int k = threadIdx.x; k < n2; k += blockDim.x) {
        const int64_t r = (int64_t)k * (m / n2);
        tw2[k] = make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]);
      }
      __syncthreads();
      const int cb1 = FFT_BUF / n1 < n2 ? FFT_BUF / n1 : n2;
      // pass 1: column DFTs (length n1) of x[n2 j1 + j2], twiddle w_m^{j2 k1}, to S[k1 n2 + j2]
      for (int j2b = 0; j2b < n2; j2b += cb1) {
        for (int u = threadIdx.x; u < cb1 * n1; u += blockDim.x) {
          const int c = u & (cb1 - 1), j1 = u / cb1;
          const int64_t jpos = (int64_t)n2 * j1 + j2b + c;
          double xa = 0.0, xb = 0.0;
          if (jpos < sd.length) {
            const int32_t p = it.pos2row[sd.offset + jpos];
            if (p >= 0) {
              xa = (double)ya[p];
              if (!isfinite(xa)) bad_a = 1.0, xa = 0.0;
              if (two) {
                xb = (double)yb[p];
                if (!isfinite(xb)) bad_b = 1.0, xb = 0.0;
              }
            }
          }
          buf[0][c * n1 + j1] = make_double2(xa, xb);
        }
        __syncthreads();
        const double2 *R = dft_lds(buf[0], buf[1], cb1, l1, tw1);
        for (int u = threadIdx.x; u < cb1 * n1; u += blockDim.x) {
          const int c = u & (cb1 - 1), k1 = u / cb1;
          const int64_t j2 = j2b + c;
          const int64_t r = (j2 * (int64_t)k1) & (m - 1);
          S[(int64_t)k1 * n2 + j2] = cmul(R[c * n1 + k1], make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]));
        }
        __threadfence_block();
        __syncthreads();
      }
      // pass 2: row DFTs (length n2), times lambda, inverse row DFTs, twiddle w_m^{-j2 k1}
      const int cb2 = FFT_BUF / n2 < n1 ? FFT_BUF / n2 : n1;
      for (int k1b = 0; k1b < n1; k1b += cb2) {
        for (int u = threadIdx.x; u < cb2 * n2; u += blockDim.x) {
          const int c = u / n2, j2 = u & (n2 - 1);
          buf[0][c * n2 + j2] = S[(int64_t)(k1b + c) * n2 + j2];
        }
        __syncthreads();
        double2 *R = dft_lds(buf[0], buf[1], cb2, l2, tw2);
        double2 *O = R == buf[0] ? buf[1] : buf[0];
        for (int u = threadIdx.x; u < cb2 * n2; u += blockDim.x) {
          const int c = u / n2, k2 = u & (n2 - 1);
          const double lam = sd.lam[(int64_t)(k1b + c) + (int64_t)n1 * k2];
          const double2 v = R[c * n2 + k2];
          O[c * n2 + k2] = make_double2(lam * v.x, -lam * v.y);  // conj(lambda X) for the inverse
        }
        __syncthreads();
        const double2 *R2 = dft_lds(O, R, cb2, l2, tw2);
        for (int u = threadIdx.x; u < cb2 * n2; u += blockDim.x) {
          const int c = u / n2, j2 = u & (n2 - 1);
          const int64_t k1 = k1b + c;
          const int64_t r = (k1 * (int64_t)j2) & (m - 1);
          // inverse row result = conj(R2); times w_m^{-j2 k1} = conj(w_m^{j2 k1}); keep conjugated
          // for the final inverse column DFT: conj(conj(R2) conj(w)) = R2 w
          S[k1 * n2 + j2] = cmul(R2[c * n2 + j2], make_double2(sd.tw[2 * r], -sd.tw[2 * r + 1]));
        }
        __threadfence_block();
        __syncthreads();
      }
      // pass 3: inverse column DFTs (length n1): (C z)_{n2 j1 + j2} = conj(DFT(conj T)) / m,
      // where S already holds conj T; results to S at the natural position n2 j1 + j2
      for (int j2b = 0; j2b < n2; j2b += cb1) {
        for (int u = threadIdx.x; u < cb1 * n1; u += blockDim.x) {
          const int c = u & (cb1 - 1), k1 = u / cb1;
          buf[0][c * n1 + k1] = S[(int64_t)k1 * n2 + j2b + c];
        }
        __syncthreads();
        const double2 *R = dft_lds(buf[0], buf[1], cb1, l1, tw1);
        for (int u = threadIdx.x; u < cb1 * n1; u += blockDim.x) {
          const int c = u & (cb1 - 1), j1 = u / cb1;
          const double2 v = R[c * n1 + j1];
          S[(int64_t)n2 * j1 + j2b + c] = make_double2(v.x * inv_m, -v.y * inv_m);
        }
        __threadfence_block();
        __syncthreads();
      }
      // residual e = h - C y0 on the segment's padded rows (0 on padding), and the dots
      for (int64_t p = sd.row0 + threadIdx.x; p < sd.row0 + sd.npad; p += blockDim.x) {
        const int32_t jg = it.idx[p];
        double va = 0.0, vb = 0.0;
        if (jg >= 0) {
          const int64_t jpos = jg - sd.offset;
          const double2 cz = S[jpos];
          const double yd = it.yd_pos[jg];
          const double xa = (double)ya[p];
          const double hva = ha[jg];
          va = hva - cz.x;
          hy_a += hva * xa;
          ydh_a += hva * yd;
          yc_a += xa * cz.x;
          if (two) {
            const double xb = (double)yb[p];
            const double hvb = hb[jg];
            vb = hvb - cz.y;
            hy_b += hvb * xb;
            ydh_b += hvb * yd;
            yc_b += xb * cz.y;
          }
        }
        ea[p] = va;
        if (two) eb[p] = vb;
      }
      __syncthreads();
    }
    const double s_hya = block_sum(hy_a, red), s_ydha = block_sum(ydh_a, red);
    const double s_yca = block_sum(yc_a, red);
    const double s_hyb = block_sum(hy_b, red), s_ydhb = block_sum(ydh_b, red);
    const double s_ycb = block_sum(yc_b, red);
    const double s_bada = block_sum(bad_a, red), s_badb = block_sum(bad_b, red);
    if (threadIdx.x == 0) {
      const double nan = __builtin_nan("");
      it.qpart[ba] = s_bada > 0 ? nan : it.qdd[0] - 2.0 * s_ydha + 2.0 * s_hya - s_yca;
      if (two) it.qpart[bb] = s_badb > 0 ? nan : it.qdd[0] - 2.0 * s_ydhb + 2.0 * s_hyb - s_ycb;
    }
  }
}

hipError_t launch_refine(const RefItem *items, const int4 *work, int64_t n_work, double *scratch,
                         int64_t scratch_per_wg, int32_t n_wg, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine, dim3((unsigned)n_wg), dim3(FFT_THREADS), 0, s, items, work, n_work,
                     (double2 *)scratch, scratch_per_wg / 2);
  return hipGetLastError();
}

}  // namespace tda
