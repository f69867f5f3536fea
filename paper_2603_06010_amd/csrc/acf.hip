// Autocovariance estimation from a stretch of strain on the device (paper Sec. II.B
// item 6: either correlate a stretch of data directly, or take a Welch PSD and its
// inverse Fourier transform; the result is truncated to the lags a segment needs).
//
// Direct:  acf[k] = (1/n) sum_{t=0}^{n-1-k} x_t x_{t+k}       (biased sample autocovariance)
// Welch:   segments s of length L starting at s L/2 (K = (n - L)/(L/2) + 1 of them), each
//          with its mean removed and multiplied by the periodic Hann window
//          w_j = (1 - cos(2 pi j / L)) / 2; with y_s the result and S2 = sum_j w_j^2,
//            acf[k] = (1/K) sum_s (1/S2) sum_{j=0}^{L-1} y_s[j] y_s[(j + k) mod L].
//          By the Wiener-Khinchin relation this is exactly the inverse DFT of the
//          two-sided mean-averaged Welch power spectral density (density scaling) times
//          the sampling rate, so it needs no FFT: the circular autocorrelations are
//          summed directly, lag tile by lag tile, the series staged through LDS in
//          chunks (one kernel for both estimators).
// Both sum in a fixed order (partial sums per chunk or segment, then in order).
#include <hip/hip_runtime.h>
#include <math.h>

#include "tda_internal.h"

namespace tda {

constexpr int ACF_LAGS = 256;                 // threads per workgroup
constexpr int ACF_PER = 8;                    // consecutive lags per thread
constexpr int ACF_TILE = ACF_LAGS * ACF_PER;  // lags per workgroup
constexpr int ACF_CHUNK = 2048;               // samples per pass through LDS
constexpr int ACF_XB = ACF_CHUNK + ACF_TILE;  // shifted samples per pass
// LDS word of shifted sample i: one pad word per 8, so that the threads' reads, 8 words
// apart, spread over the banks
__device__ __forceinline__ int acf_pad(int i) { return i + (i >> 3); }

// Sum over one series y of length L of products y[j] y[j + k] for the workgroup's lags
// k0 .. k0 + ACF_TILE - 1 and j in chunks c0 .. c0 + nc - 1 of ACF_CHUNK samples.  Thread t
// keeps the sums of the lags k0 + P t + u (u < P = ACF_PER) with y[j + P t + u] in a sliding
// window of registers: per j one read of y[j] and one of y[j + P t + P - 1] for P
// multiply-adds in independent chains.  Each lag's sum runs over j in order.  Periodic
// series (Welch segments) wrap j + k modulo L; the others read zero past the end.
//   part[(series * n_groups + group) * n_lags + k]
// grid (lag tiles, chunk groups, series); series s starts at y + s * stride
__global__ __launch_bounds__(ACF_LAGS) void k_acf_corr(const double *__restrict__ y, int64_t L,
                                                       int64_t stride, int32_t periodic,
                                                       int64_t n_lags, int32_t chunks_per_group,
                                                       double *__restrict__ part) {
  __shared__ double xa[ACF_CHUNK];
  __shared__ double xb[ACF_XB + ACF_XB / 8];
  const int64_t k0 = (int64_t)blockIdx.x * ACF_TILE;
  const double *ys = y + (int64_t)blockIdx.z * stride;
  const int64_t c_begin = (int64_t)blockIdx.y * chunks_per_group;
  const int base = ACF_PER * (int)threadIdx.x;
  double sv[ACF_PER], b[ACF_PER];
#pragma unroll
  for (int u = 0; u < ACF_PER; ++u) sv[u] = 0.0;
  for (int64_t c = c_begin; c < c_begin + chunks_per_group; ++c) {
    const int64_t j0 = c * ACF_CHUNK;
    if (j0 >= L) break;  // uniform over the workgroup
    __syncthreads();     // the previous chunk has been read
    for (int j = threadIdx.x; j < ACF_CHUNK; j += ACF_LAGS) {
      const int64_t t = j0 + j;
      xa[j] = t < L ? ys[t] : 0.0;
    }
    for (int j = threadIdx.x; j < ACF_XB; j += ACF_LAGS) {
      int64_t t = j0 + k0 + j;
      if (periodic) t %= L;
      xb[acf_pad(j)] = t < L ? ys[t] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u + 1 < ACF_PER; ++u) b[u] = xb[acf_pad(base + u)];
    for (int j = 0; j < ACF_CHUNK; ++j) {
      const double a = xa[j];
      b[ACF_PER - 1] = xb[acf_pad(j + base + ACF_PER - 1)];
#pragma unroll
      for (int u = 0; u < ACF_PER; ++u) sv[u] = fma(a, b[u], sv[u]);
#pragma unroll
      for (int u = 0; u + 1 < ACF_PER; ++u) b[u] = b[u + 1];
    }
  }
  double *out = part + ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * n_lags;
#pragma unroll
  for (int u = 0; u < ACF_PER; ++u) {
    const int64_t k = k0 + base + u;
    if (k < n_lags) out[k] = sv[u];
  }
}

// Welch segments: Y[s][j] = w_j (x[s L/2 + j] - mean_s), w the periodic Hann window.
// One workgroup per segment.
__global__ __launch_bounds__(256) void k_welch_prep(const double *__restrict__ x, int64_t L,
                                                    double *__restrict__ Y) {
  __shared__ double red[256];
  const double *xs = x + (int64_t)blockIdx.x * (L / 2);
  double m = 0.0;
  for (int64_t j = threadIdx.x; j < L; j += 256) m += xs[j];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double mean = red[0] / (double)L;
  const double c = 2.0 * M_PI / (double)L;
  double *ys = Y + (int64_t)blockIdx.x * L;
  for (int64_t j = threadIdx.x; j < L; j += 256) ys[j] = (0.5 - 0.5 * cos(c * (double)j)) * (xs[j] - mean);
}

// acf[k] = scale * sum_p part[p][k], p in order
__global__ void k_acf_sum(const double *__restrict__ part, int64_t n_parts, int64_t n_lags,
                          double scale, double *__restrict__ acf) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n_lags) return;
  double s = 0.0;
  for (int64_t c = 0; c < n_parts; ++c) s += part[c * n_lags + k];
  acf[k] = scale * s;
}

}  // namespace tda

using namespace tda;

extern "C" tda_status tda_acf_estimate(const double *x, int64_t n, int64_t n_lags, int32_t method,
                                       int64_t seg_len, double *acf, void *hip_stream) {
  if (!x || !acf) return set_error(TDA_EINVAL, "acf: NULL device pointer");
  if (n < 1 || n_lags < 1) return set_error(TDA_EINVAL, "acf: n and n_lags must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return set_error(TDA_ESTATE, "acf: not callable on a capturing stream");
  const int64_t tiles = (n_lags + ACF_TILE - 1) / ACF_TILE;
  if (tiles > 65535) return set_error(TDA_EINVAL, "acf: too many lags");
  int64_t series = 1, L = n, groups = 1, Ybytes = 0;
  int32_t cpg = 1;
  double scale = 1.0;
  if (method == TDA_ACF_DIRECT) {
    if (n_lags > n) return set_error(TDA_EINVAL, "acf: n_lags > n");
    groups = (n + ACF_CHUNK - 1) / ACF_CHUNK;  // one chunk per workgroup
    if (groups > 65535) return set_error(TDA_EINVAL, "acf: n too large for the direct estimator");
    scale = 1.0 / (double)n;
  } else if (method == TDA_ACF_WELCH) {
    if (seg_len < 2 || seg_len % 2) return set_error(TDA_EINVAL, "acf: Welch segment length must be even and >= 2");
    if (n < seg_len) return set_error(TDA_EINVAL, "acf: fewer samples than one Welch segment");
    if (n_lags > seg_len / 2) return set_error(TDA_EINVAL, "acf: n_lags > seg_len / 2");
    L = seg_len;
    series = (n - seg_len) / (seg_len / 2) + 1;
    if (series > 65535) return set_error(TDA_EINVAL, "acf: too many Welch segments");
    cpg = (int32_t)((L + ACF_CHUNK - 1) / ACF_CHUNK);  // a workgroup covers its segment
    Ybytes = series * L * (int64_t)sizeof(double);
    double s2 = 0.0;  // sum of the squared window
    for (int64_t j = 0; j < L; ++j) {
      const double w = 0.5 - 0.5 * cos(2.0 * M_PI / (double)L * (double)j);
      s2 += w * w;
    }
    scale = 1.0 / ((double)series * s2);
  } else {
    return set_error(TDA_EINVAL, "acf: unknown method");
  }
  const int64_t n_parts = series * groups;
  char *ws = nullptr;
  const size_t bytes = (size_t)Ybytes + (size_t)n_parts * n_lags * sizeof(double);
  if (hipMallocAsync((void **)&ws, bytes, s) != hipSuccess)
    return set_error(TDA_ENOMEM, "acf: workspace allocation failed");
  double *Y = (double *)ws, *part = (double *)(ws + Ybytes);
  const double *src = x;
  if (method == TDA_ACF_WELCH) {
    hipLaunchKernelGGL(k_welch_prep, dim3((unsigned)series), dim3(256), 0, s, x, L, Y);
    src = Y;
  }
  hipLaunchKernelGGL(k_acf_corr, dim3((unsigned)tiles, (unsigned)groups, (unsigned)series),
                     dim3(ACF_LAGS), 0, s, src, L, L, (int32_t)(method == TDA_ACF_WELCH), n_lags,
                     cpg, part);
  hipLaunchKernelGGL(k_acf_sum, dim3((unsigned)((n_lags + 255) / 256)), dim3(256), 0, s, part,
                     n_parts, n_lags, scale, acf);
  const hipError_t e = hipGetLastError();
  const hipError_t ef = hipFreeAsync(ws, s);
  if (e != hipSuccess) return set_error(TDA_EHIP, "acf: kernel launch failed");
  if (ef != hipSuccess) return set_error(TDA_EHIP, "acf: workspace release failed");
  return TDA_OK;
}

namespace tda {
void register_acf_attributes() {}
}  // namespace tda
