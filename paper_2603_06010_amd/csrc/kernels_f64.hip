// FP64 kernels: covariance assembly, blocked Cholesky, diagonal-block inverses,
// triangular-solve panel packing and the batched FP64 triangular solve with the
// fused sum-of-squares / log-likelihood epilogue.  gfx950 only.
//
// FP64 matrix-core operation used throughout (v_mfma_f64_16x16x4_f64):
//   D(16x16) += A(16x4) B(4x16); lane l supplies A[l%16][l/16] and B[l/16][l%16]
//   and holds D[l/16 + 4j][l%16] in register j (j = 0..3).
#include <math.h>

#include "tda_internal.h"

namespace tda {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- covariance assembly
// Dense column-major block of one segment, lower triangle only (paper Sec. II: C_ij =
// rho(|i-j|); Sec. II.B: the block of a segment restricted to its retained samples).
// Rows >= n_keep are padding: identity on the diagonal, zero elsewhere, so the
// padded factor is diag(L, I) and contributes nothing to log det or to w^T w.
__global__ void k_assemble(const double *__restrict__ acf, const int32_t *__restrict__ idx,
                           int64_t n_keep, int64_t n_pad, double *__restrict__ A) {
  const int64_t c = blockIdx.x;
  const int64_t r = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (r >= n_pad || r < c) return;
  double v;
  if (r < n_keep && c < n_keep) {
    int64_t lag = (int64_t)idx[r] - (int64_t)idx[c];
    v = acf[lag < 0 ? -lag : lag];
  } else {
    v = (r == c) ? 1.0 : 0.0;
  }
  A[c * n_pad + r] = v;
}

hipError_t launch_assemble(const double *acf, const int32_t *idx, int64_t n_keep, int64_t n_pad,
                           double *A, hipStream_t s) {
  dim3 grid((unsigned)n_pad, (unsigned)((n_pad + 255) / 256));
  hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, s, acf, idx, n_keep, n_pad, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------- blocked Cholesky
// Right-looking, panel width CP = 128, on the lower triangle of a column-major block.
// Step k: (1) factor the 128x128 diagonal block in LDS and invert it,
// (2) panel rows below: L_ik = A_ik L_kk^-T, (3) trailing update A_IJ -= L_Ik L_Jk^T.
// A pivot <= 0 or non-finite stops the factorisation: its row goes to fail[0] and
// every later kernel returns immediately.

constexpr int TS = CP + 1;  // LDS row stride (bank spread)

// The 128 x 128 diagonal block is factored in LDS by blocks of 16 columns: one wave
// factors each 16 x 16 diagonal block in registers (lane l holds row l; pivots and
// column entries come from other lanes by cross-lane reads) and inverts it (lane l
// computes column l of the inverse); then all threads solve the
// rows below against it and update the rest of the block.  The inverse X = L^-1 of the
// whole block follows by blocks of 16, X_ij = -X_ii sum_{k=j..i-1} L_ik X_kj, one block
// diagonal at a time.  X's strict lower part is kept transposed in T's strict upper part
// (X[r][c] at T[c][r]), its diagonal in diagX.
constexpr int PB = 16;                     // sub-block of the diagonal-block factorisation
constexpr int POTF2_TMP = (CP / PB - 1) * PB * PB;  // one block diagonal of the inverse

// lane `lane`'s value of v (a uniform double)
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__global__ __launch_bounds__(256) void k_potf2(double *__restrict__ A, int64_t lda, int64_t k,
                                               double *__restrict__ dinv,
                                               double *__restrict__ logdiag,
                                               int32_t *__restrict__ fail) {
  if (fail[0] >= 0) return;
  extern __shared__ double T[];  // CP x TS, then POTF2_TMP
  double *tmp = T + CP * TS;
  __shared__ double diagX[CP];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // lower triangle of the column-major block into row-major T: eight loads in flight
  // before their stores (column c = e / CP, row r = e % CP)
  for (int e0 = tid; e0 < CP * CP; e0 += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 256 * u, c = e / CP, r = e % CP;
      v[u] = r >= c ? A[(k + c) * lda + k + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 256 * u, c = e / CP, r = e % CP;
      if (r >= c) T[r * TS + c] = v[u];
    }
  }
  if (tid == 0) bad = -1;
  __syncthreads();
  for (int b0 = 0; b0 < CP; b0 += PB) {
    // (a) diagonal block: factor and invert in registers (wave 0; lane l < PB holds row l,
    // other lanes' entries come by cross-lane reads)
    if (wave == 0) {
      const int l = lane;
      const bool row = l < PB;
      double x[PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) x[c] = (row && c <= l) ? T[(b0 + l) * TS + b0 + c] : 0.0;
      int badj = -1;
#pragma unroll
      for (int j = 0; j < PB; ++j) {
        const double djj = readlane_d(x[j], j);
        if (badj < 0 && (!(djj > 0.0) || !isfinite(djj))) badj = j;
        const double piv = sqrt(djj);
        x[j] = l == j ? piv : (l > j ? x[j] / piv : x[j]);
#pragma unroll
        for (int c = j + 1; c < PB; ++c) {
          const double lcj = readlane_d(x[j], c);  // L[c][j]
          if (l >= c) x[c] -= x[j] * lcj;
        }
      }
      // column l of Y = L_bb^-1: Y[i][l] = (delta_il - sum_{q<i} L[i][q] Y[q][l]) / L[i][i]
      double y[PB];
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        double s = l == i ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) s -= readlane_d(x[q], i) * y[q];
        y[i] = s / readlane_d(x[i], i);
      }
      if (row) {
#pragma unroll
        for (int c = 0; c < PB; ++c)
          if (c <= l) T[(b0 + l) * TS + b0 + c] = x[c];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
          if (i == l) diagX[b0 + l] = y[i];
          if (i > l) T[(b0 + l) * TS + b0 + i] = y[i];
        }
      }
      if (l == 0 && badj >= 0) bad = b0 + badj;
    }
    __syncthreads();
    if (bad >= 0) break;
    // (b) rows below within the block: X_r = A_r L_bb^-T,
    // X_r[c] = A_r[c] Y[c][c] + sum_{q<c} A_r[q] Y[c][q], Y[c][q] at T[b0+q][b0+c]
    const int nrow = CP - b0 - PB;
    const int nout = nrow * PB;
    double res[12];
#pragma unroll
    for (int u = 0; u < 12; ++u) {
      const int e = tid + 256 * u;
      res[u] = 0.0;
      if (e < nout) {
        const int r = b0 + PB + e / PB, c = e % PB;
        const double *Ar = T + r * TS + b0;
        double a4[4] = {Ar[c] * diagX[b0 + c], 0.0, 0.0, 0.0};
        int q = 0;
        for (; q + 3 < c; q += 4) {
#pragma unroll
          for (int v = 0; v < 4; ++v) a4[v] += Ar[q + v] * T[(b0 + q + v) * TS + b0 + c];
        }
        for (; q < c; ++q) a4[0] += Ar[q] * T[(b0 + q) * TS + b0 + c];
        res[u] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 12; ++u) {
      const int e = tid + 256 * u;
      if (e < nout) T[(b0 + PB + e / PB) * TS + b0 + e % PB] = res[u];
    }
    __syncthreads();
    // (c) trailing update of the block: T[r][c] -= X_r . X_c for b0+PB <= c <= r
    const int ntri = nrow * (nrow + 1) / 2;
    for (int e = tid; e < ntri; e += 256) {
      int rr = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while (rr * (rr + 1) / 2 > e) --rr;
      while ((rr + 1) * (rr + 2) / 2 <= e) ++rr;
      const int cc = e - rr * (rr + 1) / 2;
      const int r = b0 + PB + rr, c = b0 + PB + cc;
      const double *Xr = T + r * TS + b0, *Xc = T + c * TS + b0;
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < PB; ++q) a4[q & 3] += Xr[q] * Xc[q];
      T[r * TS + c] -= (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    __syncthreads();
  }
  if (bad >= 0) {
    if (tid == 0) fail[0] = (int32_t)(k + bad);
    return;
  }
  // L back to global (lower, incl. diagonal)
  for (int e0 = tid; e0 < CP * CP; e0 += 8 * 256) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 256 * u, c = e / CP, r = e % CP;
      if (r >= c) A[(k + c) * lda + k + r] = T[r * TS + c];
    }
  }
  // off-diagonal blocks of X = L^-1, one block diagonal (distance dd) at a time, one
  // 16 x 16 block per wave and FP64 matrix-core op: tmp_ij = sum_{kb=j..i-1} L_i,kb X_kb,j,
  // then X_ij = -Y_ii tmp_ij.  Operand lane l supplies row l % 16 and k-index l / 16 of
  // the k-step; X[R][C] (R > C) is read at T[C][R], its diagonal from diagX, zero above.
  {
    const int lr = lane & 15, lk = lane >> 4;
    auto xat = [&](int R, int C) -> double {
      return R > C ? T[C * TS + R] : (R == C ? diagX[R] : 0.0);
    };
    for (int dd = 1; dd < CP / PB; ++dd) {
      const int nb = CP / PB - dd;
      for (int bi = wave; bi < nb; bi += 4) {
        const int i = bi + dd, j = bi;
        d4 acc = d4{0, 0, 0, 0};
        for (int kb = j; kb < i; ++kb)
#pragma unroll
          for (int s4 = 0; s4 < PB; s4 += 4) {
            const int K = PB * kb + s4 + lk;
            const double a = T[(PB * i + lr) * TS + K];
            const double bv = xat(K, PB * j + lr);
            acc = mfma64(a, bv, acc);
          }
        // D[q][n] at lane (q % 4) * 16 + n, register q / 4
#pragma unroll
        for (int u = 0; u < 4; ++u) tmp[bi * PB * PB + (lk + 4 * u) * PB + lr] = acc[u];
      }
      __syncthreads();
      for (int bi = wave; bi < nb; bi += 4) {
        const int i = bi + dd, j = bi, R0 = PB * i;
        d4 acc = d4{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < PB; s4 += 4) {
          const double a = xat(R0 + lr, R0 + s4 + lk);             // Y_ii[r][q]
          const double bv = tmp[bi * PB * PB + (s4 + lk) * PB + lr];  // tmp[q][c]
          acc = mfma64(a, bv, acc);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) T[(PB * j + lr) * TS + R0 + lk + 4 * u] = -acc[u];
      }
      __syncthreads();
    }
  }
  // dinv[t*CP + c] = X[c][t]  (row t of X^T)
  for (int e = tid; e < CP * CP; e += 256) {
    const int t = e / CP, c = e % CP;
    double v = 0.0;
    if (c > t) v = T[t * TS + c];
    else if (c == t) v = diagX[t];
    dinv[e] = v;
  }
  if (wave == 0) {
    double s = log(T[lane * TS + lane]) + log(T[(lane + 64) * TS + lane + 64]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) logdiag[0] = s;
  }
}

// rows i in [k+CP, n): L[i, k:k+CP] = A[i, k:k+CP] * X^T, X = L_kk^-1; 64 rows per workgroup.
__global__ __launch_bounds__(256) void k_panel(double *__restrict__ A, int64_t lda, int64_t k,
                                               const double *__restrict__ dinvT,
                                               const int32_t *__restrict__ fail) {
  if (fail[0] >= 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane >> 4, lc = lane & 15;
  const int64_t i0 = k + CP + (int64_t)blockIdx.x * 64 + 16 * w;
  d4 acc[8];
#pragma unroll
  for (int ct = 0; ct < 8; ++ct) acc[ct] = d4{0, 0, 0, 0};
  // operands in batches of TG k-steps of 4, each batch fetched one batch ahead of its
  // products (two register buffers), so that the loads of a batch wait once
  constexpr int TG = 4, NB = CP / (4 * TG);
  static_assert(NB % 2 == 0, "whole buffer pairs");
  double av[2][TG], bv[2][TG][8];
  auto fetch = [&](int buf, int g) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < TG; ++u) {
      const int t0 = 4 * (g * TG + u);
      av[buf][u] = A[(k + t0 + lr) * lda + i0 + lc];
#pragma unroll
      for (int ct = 0; ct < 8; ++ct) bv[buf][u][ct] = dinvT[(t0 + lr) * CP + 16 * ct + lc];
    }
  };
  auto consume = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < TG; ++u)
#pragma unroll
      for (int ct = 0; ct < 8; ++ct) acc[ct] = mfma64(av[buf][u], bv[buf][u][ct], acc[ct]);
  };
  fetch(0, 0);
  for (int g = 0; g < NB; g += 2) {
    fetch(1, g + 1);
    consume(0);
    if (g + 2 < NB) fetch(0, g + 2);
    consume(1);
  }
#pragma unroll
  for (int ct = 0; ct < 8; ++ct)
#pragma unroll
    for (int j = 0; j < 4; ++j) A[(k + 16 * ct + lc) * lda + i0 + lr + 4 * j] = acc[ct][j];
}

// Trailing update A_IJ -= L_I,K L_J,K^T over panel columns K = [kcol, kcol + kw) of the
// region from row/column r0 in lower 128 x 128 tiles (I >= J, tile I covers rows
// r0 + 128 I ..): the 128 rows x 16 columns of both operands per step are staged in LDS
// (double-buffered, one chunk loaded into registers while the previous one is multiplied).
// Four waves each take a 64 x 64 quarter as 4 x 4 FP64 matrix-core tiles, with the MFMA's
// fast index on C's rows so that the read-modify-write of C is coalesced.
// col_only != 0: the tiles of tile column jb only (I = jb + blockIdx.x); else the lower
// triangle of tiles from (jb, jb).
constexpr int SY = 128;       // tile edge
constexpr int SK = 16;        // panel columns per LDS stage
constexpr int SYP = SY + 16;  // LDS row stride (bank spread between the four k rows)

__global__ __launch_bounds__(256, 2) void k_syrk(double *__restrict__ A, int64_t lda, int64_t kcol,
                                                 int32_t kw, int64_t r0, int32_t jb,
                                                 int32_t col_only,
                                                 const int32_t *__restrict__ fail) {
  if (fail[0] >= 0) return;
  __shared__ double Ls[2][2][SK][SYP];  // [buffer][I or J panel rows][column][row]
  const int64_t e = blockIdx.x;
  int64_t I, J;
  if (col_only) {
    J = jb;
    I = jb + e;
  } else {
    int64_t t = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while (t * (t + 1) / 2 > e) --t;
    while ((t + 1) * (t + 2) / 2 <= e) ++t;
    I = jb + t;
    J = jb + e - t * (t + 1) / 2;
  }
  const int64_t I0 = r0 + SY * I, J0 = r0 + SY * J;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;  // rows I0 + 64 wr .., columns J0 + 64 wc ..
  const int lr = lane >> 4, lc = lane & 15;
  // staging: pair p = tid + 256 u (u < 8) of (which, column t, rows 2q and 2q + 1)
  typedef double d2 __attribute__((ext_vector_type(2)));
  d2 stage[8];
  auto load_chunk = [&](int c) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int p = tid + 256 * u;
      const int which = p >> 10, t = (p >> 6) & (SK - 1), q = p & 63;
      const int64_t row0 = which ? J0 : I0;
      stage[u] = *(const d2 *)(A + (kcol + SK * c + t) * lda + row0 + 2 * q);
    }
  };
  auto store_chunk = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int p = tid + 256 * u;
      const int which = p >> 10, t = (p >> 6) & (SK - 1), q = p & 63;
      *(d2 *)&Ls[buf][which][t][2 * q] = stage[u];
    }
  };
  d4 acc[4][4];  // [J group of 16][I group of 16]: D[m][n] = C[I row n][J column m]
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = d4{0, 0, 0, 0};
  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  const int NCH = kw / SK;
  for (int c = 0; c < NCH; ++c) {
    const int buf = c & 1;
    if (c + 1 < NCH) load_chunk(c + 1);
#pragma unroll
    for (int t0 = 0; t0 < SK; t0 += 4) {
      double a[4], b[4];
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) a[mi] = Ls[buf][1][t0 + lr][64 * wc + 16 * mi + lc];
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) b[ni] = Ls[buf][0][t0 + lr][64 * wr + 16 * ni + lc];
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = mfma64(a[mi], b[ni], acc[mi][ni]);
    }
    if (c + 1 < NCH) store_chunk(buf ^ 1);
    __syncthreads();
  }
  // C[r][cc] -= acc, r = I0 + 64 wr + 16 ni + lc, cc = J0 + 64 wc + 16 mi + lr + 4 j; lower part only
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t r = I0 + 64 * wr + 16 * ni + lc;
        const int64_t cc = J0 + 64 * wc + 16 * mi + lr + 4 * j;
        if (I != J || r >= cc) A[cc * lda + r] -= acc[mi][ni][j];
      }
}

// One segment's factorisation, two 128-column panels per outer step: panel 2s (diagonal
// block and rows below), its update of the next 128 columns, panel 2s + 1, then one
// trailing update of everything beyond with both panels (K = 256, half the read-modify-
// write traffic of K = 128).  Look-ahead over two streams: stream a runs the panels, the
// first 128 columns of each trailing update and the next outer step's panels while
// stream b runs the rest of the trailing update; a waits for b's previous update before
// it touches the columns that update wrote.
hipError_t launch_cholesky(double *A, int64_t n, double *dinv, double *logdiag, int32_t *fail,
                           hipStream_t s) {
  const size_t lds = sizeof(double) * (CP * TS + POTF2_TMP);
  hipStream_t sa = nullptr, sb = nullptr;
  hipEvent_t e0 = nullptr, ea = nullptr, eb = nullptr;
  hipError_t err = hipSuccess;
  bool b_pending = false;  // eb marks an update on b that a has not waited for
  auto chk = [&](hipError_t x) {
    if (err == hipSuccess && x != hipSuccess) err = x;
    return err == hipSuccess;
  };
  auto diag_and_panel = [&](int64_t k) {
    hipLaunchKernelGGL(k_potf2, dim3(1), dim3(256), lds, sa, A, n, k, dinv + (k / CP) * CP * CP,
                       logdiag + k / CP, fail);
    const int64_t rest = n - k - CP;
    if (rest > 0)
      hipLaunchKernelGGL(k_panel, dim3((unsigned)(rest / 64)), dim3(256), 0, sa, A, n, k,
                         dinv + (k / CP) * CP * CP, fail);
    return chk(hipGetLastError());
  };
  if (chk(hipStreamCreateWithFlags(&sa, hipStreamNonBlocking)) &&
      chk(hipStreamCreateWithFlags(&sb, hipStreamNonBlocking)) &&
      chk(hipEventCreateWithFlags(&e0, hipEventDisableTiming)) &&
      chk(hipEventCreateWithFlags(&ea, hipEventDisableTiming)) &&
      chk(hipEventCreateWithFlags(&eb, hipEventDisableTiming)) && chk(hipEventRecord(e0, s)) &&
      chk(hipStreamWaitEvent(sa, e0, 0)) && chk(hipStreamWaitEvent(sb, e0, 0))) {
    // n is a multiple of 2 CP (segments are padded to 256 rows)
    for (int64_t k = 0; k < n && err == hipSuccess; k += 2 * CP) {
      diag_and_panel(k);
      // the next 128 columns need b's last update (it covered them) and panel k
      if (b_pending) chk(hipStreamWaitEvent(sa, eb, 0));
      b_pending = false;
      const int64_t T1 = (n - k - CP) / SY;
      hipLaunchKernelGGL(k_syrk, dim3((unsigned)T1), dim3(256), 0, sa, A, n, k, CP, k + CP, 0, 1,
                         fail);
      diag_and_panel(k + CP);
      const int64_t r0 = k + 2 * CP, T = (n - r0) / SY;
      if (T <= 0) break;
      chk(hipEventRecord(ea, sa));  // both panels finished
      if (T > 1) {
        chk(hipStreamWaitEvent(sb, ea, 0));
        hipLaunchKernelGGL(k_syrk, dim3((unsigned)((T - 1) * T / 2)), dim3(256), 0, sb, A, n, k,
                           2 * CP, r0, 1, 0, fail);
        chk(hipEventRecord(eb, sb));
        b_pending = true;
      }
      hipLaunchKernelGGL(k_syrk, dim3((unsigned)T), dim3(256), 0, sa, A, n, k, 2 * CP, r0, 0, 1,
                         fail);
      chk(hipGetLastError());
    }
    chk(hipEventRecord(ea, sa));
    chk(hipEventRecord(eb, sb));
    chk(hipStreamWaitEvent(s, ea, 0));
    chk(hipStreamWaitEvent(s, eb, 0));
  }
  // the caller synchronises right after the factorisation anyway
  if (sa) (void)hipStreamSynchronize(sa), (void)hipStreamDestroy(sa);
  if (sb) (void)hipStreamSynchronize(sb), (void)hipStreamDestroy(sb);
  if (e0) (void)hipEventDestroy(e0);
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  return err;
}

// ---------------------------------------------------------------- inverses of TB x TB diagonal blocks
// inv([Ai^-1 0; B C]) with the two CP x CP Cholesky inverses:
//   [Ai 0; X21 Ci], X21 = -Ci B Ai.  Output row-major TB x TB (upper part zero).
__global__ __launch_bounds__(256) void k_diag_inverse(const double *__restrict__ A, int64_t lda,
                                                      const double *__restrict__ dinv128,
                                                      double *__restrict__ out) {
  extern __shared__ double T1[];  // CP x TS : B * Ai
  const int b = blockIdx.x;
  const int64_t r0 = (int64_t)b * TB;
  const double *dA = dinv128 + (int64_t)(2 * b) * CP * CP;      // dA[t*CP + c] = Ai[c][t]
  const double *dC = dinv128 + (int64_t)(2 * b + 1) * CP * CP;  // dC[t*CP + c] = Ci[c][t]
  double *O = out + (int64_t)b * TB * TB;
  const int tid = threadIdx.x;
  // T1[r][c] = sum_{t >= c} B[r][t] Ai[t][c],  B[r][t] = L[r0+CP+r][r0+t]
  for (int e = tid; e < CP * CP; e += 256) {
    const int r = e % CP, c = e / CP;
    double s = 0.0;
    for (int t = c; t < CP; ++t) s += A[(r0 + t) * lda + r0 + CP + r] * dA[c * CP + t];
    T1[r * TS + c] = s;
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    double v = 0.0;
    if (r < CP) {
      if (c < CP && c <= r) v = dA[c * CP + r];
    } else if (c < CP) {
      const int rr = r - CP;
      double s = 0.0;
      for (int t = 0; t <= rr; ++t) s += dC[t * CP + rr] * T1[t * TS + c];
      v = -s;
    } else {
      const int rr = r - CP, cc = c - CP;
      if (cc <= rr) v = dC[cc * CP + rr];
    }
    O[e] = v;
  }
}

hipError_t launch_diag_inverse(const double *A, int64_t n, const double *dinv128, double *dinv256,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_diag_inverse, dim3((unsigned)(n / TB)), dim3(256),
                     sizeof(double) * CP * TS, s, A, n, dinv128, dinv256);
  return hipGetLastError();
}

// ---------------------------------------------------------------- panel packing
// Block row i (TB rows) of a segment owns K_i = i*TB off-diagonal columns and TB
// diagonal-inverse columns.  Layout [s][t][lane]: k-step s (4 columns), row tile t
// (16 rows), lane l holds row 16t + l%16, column 4s + l/16 -- exactly the A operand
// of the FP64 matrix-core op.  Off-diagonal entries are stored negated so the solve
// accumulates with plain multiply-adds.
__global__ void k_pack(const double *__restrict__ A, int64_t lda, const double *__restrict__ dinv256,
                       double *__restrict__ panels, const int64_t *__restrict__ offs, int32_t blk0) {
  const int i = blockIdx.y;  // local block row
  const int64_t K = (int64_t)i * TB;
  const int64_t total = (K + TB) * TB;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int lane = (int)(e & 63), t = (int)((e >> 6) & 15);
  const int64_t s = e >> 10;
  const int64_t row = 16 * t + (lane & 15);
  const int64_t col = 4 * s + (lane >> 4);
  double v;
  if (col < K)
    v = -A[col * lda + K + row];
  else
    v = dinv256[(int64_t)i * TB * TB + row * TB + (col - K)];
  panels[offs[blk0 + i] + e] = v;
}

hipError_t launch_pack_panels(const double *A, int64_t n, int64_t row0, const double *dinv256,
                              double *panels, const int64_t *panel_off_dev, int32_t blk0,
                              int32_t nblk_seg, hipStream_t s) {
  (void)row0;
  const int64_t maxel = (int64_t)nblk_seg * TB * TB;
  dim3 grid((unsigned)((maxel + 255) / 256), (unsigned)nblk_seg);
  hipLaunchKernelGGL(k_pack, grid, dim3(256), 0, s, A, n, dinv256, panels, panel_off_dev, blk0);
  return hipGetLastError();
}

__global__ void k_sum_logdet(const double *logdiag, int64_t count, double *logdet) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int64_t i = 0; i < count; ++i) s += logdiag[i];
    logdet[0] = 2.0 * s;
  }
}

hipError_t launch_sum_logdet(const double *logdiag, int64_t count, double *logdet, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_logdet, dim3(1), dim3(64), 0, s, logdiag, count, logdet);
  return hipGetLastError();
}

// ---------------------------------------------------------------- batched FP64 triangular solve
// One workgroup solves L W = R for 32 right-hand sides (columns c0..c0+31) over the block
// rows [blk_begin, blk_end), left-looking (paper Sec. III.A, the CDL solve):
//   acc = R_i + sum_{j<i} (-L_ij) W_j      (FP64 matrix cores, panel streamed from HBM/L2)
//   W_i = inv(L_ii) acc                    (acc staged in LDS)
// Four waves; wave w owns the 16-row tiles w, w+4, w+8, w+12 of each block row, so the
// triangular diagonal product is balanced.  Solved rows go to the tile's scratch and are
// re-read by later block rows.  MODE_LOGLIK fuses R = d - h_b on the retained rows and
// the epilogue out[b] = -1/2 sum_i W[i][b]^2 + cterm (eq:td_like_whitened plus the
// constant); MODE_IDENTITY solves against identity columns (W = L^-1).
__device__ __forceinline__ void trsm_tile(const TrsmItem &it, const TrsmTile &tl) {
  __shared__ double S[TB * BC];
  __shared__ double red[4][4][BC];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane >> 4, lc = lane & 15;
  double *W = it.scratch + tl.w_off;
  const int64_t rbase = (int64_t)tl.blk_begin * TB;
  double ss0 = 0.0, ss1 = 0.0;

  for (int i = tl.blk_begin; i < tl.blk_end; ++i) {
    d4 acc[4][2];
    const int64_t rowblk = (int64_t)i * TB;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = w + 4 * j;
#pragma unroll
      for (int tc = 0; tc < 2; ++tc) {
        const int col = 16 * tc + lc;
        const int b = tl.c0 + col;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = rowblk + 16 * t + lr + 4 * v;
          double val = 0.0;
          if (it.mode == MODE_LOGLIK) {
            const int32_t p = it.idx[row];
            if (p >= 0 && b < it.B) val = it.d[p] - template_row(it, b)[p];
          } else {
            val = (row == (int64_t)b) ? 1.0 : 0.0;
          }
          acc[j][tc][v] = val;
        }
      }
    }
    const double *P = it.panels + it.panel_off[i];
    const int bf = it.blk_first[i];
    const int f = bf > tl.blk_begin ? bf : tl.blk_begin;
    const int s_begin = (f - bf) * (TB / 4);
    const int s_end = (i - bf) * (TB / 4);
    const double *Wk = W + ((int64_t)f * TB - rbase) * BC;
    // Operands of GK k-steps are fetched NBUF - 1 groups ahead of the matrix cores (NBUF
    // register buffers in a ring), so the loads of a group have that many groups of products
    // to arrive.  The k-range of a block row is a multiple of 64 k-steps, so groups tile it
    // exactly; no fetch goes past it.
    constexpr int GK = 4, NBUF = 6;
    double pa[NBUF][GK][4], pb[NBUF][GK][2];
    auto fetch = [&](int bsel, int s0) {
#pragma unroll
      for (int kk = 0; kk < GK; ++kk) {
        const double *Ps = P + (int64_t)(s0 + kk) * 16 * 64 + lane;
#pragma unroll
        for (int j = 0; j < 4; ++j) pa[bsel][kk][j] = Ps[(w + 4 * j) * 64];
        const double *Wr = Wk + ((int64_t)(s0 + kk - s_begin) * 4 + lr) * BC + lc;
        pb[bsel][kk][0] = Wr[0];
        pb[bsel][kk][1] = Wr[16];
      }
    };
    auto consume = [&](int bsel) {
#pragma unroll
      for (int kk = 0; kk < GK; ++kk)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[j][0] = mfma64(pa[bsel][kk][j], pb[bsel][kk][0], acc[j][0]);
          acc[j][1] = mfma64(pa[bsel][kk][j], pb[bsel][kk][1], acc[j][1]);
        }
    };
    if (s_begin < s_end) {
#pragma unroll
      for (int u = 0; u < NBUF - 1; ++u)
        if (s_begin + u * GK < s_end) fetch(u, s_begin + u * GK);
      // group s + u GK sits in buffer u
      for (int s = s_begin; s < s_end; s += NBUF * GK) {
#pragma unroll
        for (int u = 0; u < NBUF; ++u) {
          if (s + u * GK >= s_end) break;
          const int ahead = s + (u + NBUF - 1) * GK;
          if (ahead < s_end) fetch((u + NBUF - 1) % NBUF, ahead);
          consume(u);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int tc = 0; tc < 2; ++tc)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          S[(16 * (w + 4 * j) + lr + 4 * v) * BC + 16 * tc + lc] = acc[j][tc][v];
    __syncthreads();
    double *Wi = W + (rowblk - rbase) * BC;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = w + 4 * j;
      d4 x0 = {0, 0, 0, 0}, x1 = {0, 0, 0, 0};
      const double *Pd = P + (int64_t)s_end * 16 * 64 + t * 64 + lane;
#pragma unroll 8
      for (int s2 = 0; s2 < 4 * (t + 1); ++s2) {
        const double a = Pd[(int64_t)s2 * 16 * 64];
        const double *Sr = S + (4 * s2 + lr) * BC + lc;
        x0 = mfma64(a, Sr[0], x0);
        x1 = mfma64(a, Sr[16], x1);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = 16 * t + lr + 4 * v;
        Wi[r * BC + lc] = x0[v];
        Wi[r * BC + 16 + lc] = x1[v];
        ss0 += x0[v] * x0[v];
        ss1 += x1[v] * x1[v];
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  if (it.mode == MODE_LOGLIK) {
    red[w][lr][lc] = ss0;
    red[w][lr][16 + lc] = ss1;
    __syncthreads();
    if (threadIdx.x < BC) {
      const int col = threadIdx.x;
      double q = 0.0;
      for (int w2 = 0; w2 < 4; ++w2)
        for (int r2 = 0; r2 < 4; ++r2) q += red[w2][r2][col];
      const int b = tl.c0 + col;
      if (b < it.B) it.out[b] = -0.5 * q + it.cterm;
    }
  }
}

__global__ __launch_bounds__(256, 1) void k_trsm_f64(const TrsmItem *__restrict__ items,
                                                     const TrsmTile *__restrict__ tiles) {
  const TrsmTile tl = tiles[blockIdx.x];
  const TrsmItem it = items[tl.item];
  trsm_tile(it, tl);
}

hipError_t launch_trsm_f64(const TrsmItem *items, const TrsmTile *tiles, int64_t n_tiles,
                           hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_f64, dim3((unsigned)n_tiles), dim3(256), 0, s, items, tiles);
  return hipGetLastError();
}

// One workgroup per (column tile, 64-row chunk), chunks fastest; 256 threads: 64 rows x
// 4 column groups, 8 columns each.  Writes run along the rows of one template
// (coalesced); the reads of a row's 32 templates share cache lines across the groups.
__global__ __launch_bounds__(256) void k_whiten_export(const double *__restrict__ scratch,
                                                       const int32_t *__restrict__ retpos,
                                                       int64_t n_pad, int64_t n_chunks,
                                                       int64_t B, double *__restrict__ wres,
                                                       int64_t ldw) {
  const int64_t t = blockIdx.x / n_chunks;
  const int64_t r = (blockIdx.x % n_chunks) * 64 + (threadIdx.x & 63);
  const int cg = threadIdx.x >> 6;
  if (r >= n_pad) return;
  const int32_t pos = retpos[r];
  if (pos < 0) return;
  const double *src = scratch + (t * n_pad + r) * BC;
#pragma unroll
  for (int i = 0; i < BC / 4; ++i) {
    const int c = cg + 4 * i;
    const int64_t b = t * BC + c;
    if (b < B) wres[b * ldw + pos] = src[c];
  }
}

hipError_t launch_whiten_export(const double *scratch, const int32_t *retpos, int64_t n_pad,
                                int64_t B, double *wres, int64_t ldw, hipStream_t s) {
  const int64_t nt = (B + BC - 1) / BC, nc = (n_pad + 63) / 64;
  if (nt <= 0 || nc <= 0) return hipSuccess;
  if (nt * nc > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_whiten_export, dim3((unsigned)(nt * nc)), dim3(256), 0, s, scratch, retpos,
                     n_pad, nc, B, wres, ldw);
  return hipGetLastError();
}

// One item passed by value; tile t covers columns [32t, 32t+32) over all block rows.
__global__ __launch_bounds__(256, 1) void k_trsm_f64_single(const TrsmItem it, int32_t nblk) {
  const TrsmTile tl{0, (int32_t)(blockIdx.x * BC), 0, nblk,
                    (int64_t)blockIdx.x * (int64_t)nblk * TB * BC};
  trsm_tile(it, tl);
}

hipError_t launch_trsm_f64_single(const TrsmItem &it, int32_t nblk, int64_t n_tiles,
                                  hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_f64_single, dim3((unsigned)n_tiles), dim3(256), 0, s, it, nblk);
  return hipGetLastError();
}

void register_kernel_attributes() {
  register_mixed_attributes();
  register_acf_attributes();
  hipFuncSetAttribute((const void *)k_potf2, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)(sizeof(double) * (CP * TS + POTF2_TMP)));
  hipFuncSetAttribute((const void *)k_diag_inverse, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)(sizeof(double) * CP * TS));
}

// ---------------------------------------------------------------- explicit-inverse (CDO) FP64 form
// Residual rows per template: R[b][r] = d[idx[r]] - h_b[idx[r]] on retained rows, 0 on
// padding rows and on the padded templates b >= B.  grid (n_pad / 256, <= 65535), the
// templates strided over grid.y
__global__ void k_cdo_pack(const CdoItem *__restrict__ items) {
  const CdoItem &it = items[0];
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= it.n_pad) return;
  const int32_t p = it.idx[r];
  for (int64_t b = blockIdx.y; b < it.Bp; b += gridDim.y) {
    double v = 0.0;
    if (b < it.B && p >= 0) v = it.d[p] - it.H[b * it.ldh + p];
    it.R[b * it.n_pad + r] = v;
  }
}

hipError_t launch_cdo_pack(const CdoItem *it_dev, const CdoItem &it, hipStream_t s) {
  dim3 grid((unsigned)((it.n_pad + 255) / 256), (unsigned)(it.Bp < 65535 ? it.Bp : 65535));
  hipLaunchKernelGGL(k_cdo_pack, grid, dim3(256), 0, s, it_dev);
  return hipGetLastError();
}

// One 16-column group of the K loop: every lane loads four consecutive columns of its row
// of W (A) and of its template's residual (B).  Matrix-core k-step j of the group takes
// column 16 q + 4 g + j from lane group g = lane / 16, for A and B alike; the order of
// the columns inside the sum is the only thing this permutes.
struct CdoStep {
  d4 a[4], b[4];
};

// w[rows of block i][templates T0 .. T0 + 63] over the 16-column groups q of [q0, q0 + nq)
// (walked downwards when dir < 0), four waves of 64 rows x 64 templates.
__device__ __forceinline__ void cdo_block(const CdoItem &it, int i, int64_t T0, int dir,
                                          double *partrow) {
  __shared__ double red[4][CDO_T];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, lc = lane & 15;
  const int bf = it.blk_first[i];
  const int64_t q0 = (int64_t)bf * (TB / 16), nq = (int64_t)(i + 1 - bf) * (TB / 16);
  const int64_t row0 = (int64_t)i * TB + 64 * w + lc;
  const double *Rb = it.R + (T0 + lc) * it.n_pad + 4 * g;
  auto load = [&](int64_t k, CdoStep &st) __attribute__((always_inline)) {
    const int64_t kk = k < nq ? k : nq - 1;
    const int64_t q = dir > 0 ? q0 + kk : q0 + nq - 1 - kk;
    const int64_t ct = q >> 1;
    const double *Wt = it.w64 + it.w64_off[ct] + 16 * (q & 1) + 4 * g;
    const int64_t rb = it.w64_rb[ct];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      st.a[t] = *(const d4 *)(Wt + (row0 + 16 * t - rb) * 32);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      st.b[c] = *(const d4 *)(Rb + (int64_t)16 * c * it.n_pad + 16 * q);
  };
  d4 acc[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[t][c] = d4{0, 0, 0, 0};
  CdoStep st[3];
  load(0, st[0]);
  load(1, st[1]);
  int64_t k = 0;
  for (; k + 3 <= nq; k += 3) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      load(k + u + 2, st[(u + 2) % 3]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[t][c] = mfma64(st[u].a[t][j], st[u].b[c][j], acc[t][c]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // the K range is a multiple of 16 groups: 0, 1 or 2 groups remain, in the first stages
#pragma unroll
  for (int u = 0; u < 2; ++u)
    if (k + u < nq)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            acc[t][c] = mfma64(st[u].a[t][j], st[u].b[c][j], acc[t][c]);
  // per template: sum of squares over the wave's 64 rows (lanes g = 0..3 of a column hold
  // four rows each of every 16-row tile), then over the four waves in LDS
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double ss = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) ss += acc[t][c][v] * acc[t][c][v];
    ss += __shfl_xor(ss, 16);
    ss += __shfl_xor(ss, 32);
    if (g == 0) red[w][16 * c + lc] = ss;
  }
  __syncthreads();
  if (threadIdx.x < CDO_T)
    partrow[T0 + threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] +
                                red[2][threadIdx.x] + red[3][threadIdx.x];
  __syncthreads();
}

// Work entries (item 0, block, template group of 64, 0): block l of a segment and its
// partner nb - 1 - l, the second with K walked downwards (as the BF16x3 products).
__global__ __launch_bounds__(256, 1) void k_cdo(const CdoItem *__restrict__ items,
                                                const int4 *__restrict__ work) {
  const int4 wk = work[blockIdx.x];
  if (wk.y < 0) return;
  const CdoItem &it = items[wk.x];
  const int64_t T0 = (int64_t)wk.z * CDO_T;
  const int partner = it.blk_first[wk.y] + it.blk_last[wk.y] - wk.y;
  cdo_block(it, wk.y, T0, 1, it.part + (int64_t)wk.y * it.Bp);
  if (partner != wk.y) cdo_block(it, partner, T0, -1, it.part + (int64_t)partner * it.Bp);
}

hipError_t launch_cdo(const CdoItem *it_dev, const int4 *work, int64_t n_work, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cdo, dim3((unsigned)n_work), dim3(256), 0, s, it_dev, work);
  return hipGetLastError();
}

// out[b] = -1/2 sum_i part[i][b] + cterm, blocks in order
__global__ void k_cdo_finish(const CdoItem *__restrict__ items, int64_t B) {
  const CdoItem &it = items[0];
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  double q = 0.0;
  for (int i = 0; i < it.nblk; ++i) q += it.part[(int64_t)i * it.Bp + b];
  it.out[b] = -0.5 * q + it.cterm;
}

hipError_t launch_cdo_finish(const CdoItem *it_dev, int64_t B, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cdo_finish, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, it_dev, B);
  return hipGetLastError();
}

// ---------------------------------------------------------------- network sums
// out_g[b] = sum over the items of group g (in item order) of parts_item[b].
__global__ void k_combine(const double *__restrict__ parts, const int64_t *__restrict__ part_off,
                          const int32_t *__restrict__ group_of, int64_t n_items,
                          double *const *__restrict__ outs, const int64_t *__restrict__ Bs) {
  const int g = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= Bs[g]) return;
  double s = 0.0;
  for (int64_t it = 0; it < n_items; ++it)
    if (group_of[it] == g) s += parts[part_off[it] + b];
  outs[g][b] = s;
}

hipError_t launch_combine(const double *parts, const int64_t *part_off, const int32_t *group_of,
                          int64_t n_items, double *const *outs, const int64_t *Bs,
                          int64_t n_groups, int64_t max_B, hipStream_t s) {
  if (n_groups <= 0 || max_B <= 0) return hipSuccess;
  dim3 grid((unsigned)((max_B + 255) / 256), (unsigned)n_groups);
  hipLaunchKernelGGL(k_combine, grid, dim3(256), 0, s, parts, part_off, group_of, n_items, outs, Bs);
  return hipGetLastError();
}

// Copy result runs: desc[3k] = destination pointer (as integer), desc[3k+1] = source
// offset, desc[3k+2] = count.
__global__ void k_scatter(const int64_t *__restrict__ desc, const double *__restrict__ src) {
  const int64_t k = blockIdx.x;
  double *dst = reinterpret_cast<double *>(desc[3 * k]);
  const int64_t off = desc[3 * k + 1], cnt = desc[3 * k + 2];
  for (int64_t j = threadIdx.x; j < cnt; j += blockDim.x) dst[j] = src[off + j];
}

hipError_t launch_scatter(const int64_t *desc, int64_t n, const double *src, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)n), dim3(64), 0, s, desc, src);
  return hipGetLastError();
}

// Inner products from three log-likelihoods with the same constant c: an evaluation
// against the data (out), one against zero data (hh: logL = c - <h,h>/2) and one of the
// data against a zero template (dd: logL = c - <d,d>/2).  From q = <d,d> - 2 <d,h> + <h,h>
// with q = -2 (logL - c): <h,h> = -2 (hh - c) and <d,h> = out - dd + <h,h>/2.  hh is
// overwritten with <h,h>; dh may be NULL.
__global__ void k_terms_combine(const double *__restrict__ out, double *__restrict__ hh,
                                const double *__restrict__ dd, double cterm, int64_t B,
                                double *__restrict__ dh) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const double v = -2.0 * (hh[b] - cterm);
  hh[b] = v;
  if (dh) dh[b] = out[b] - dd[0] + 0.5 * v;
}

hipError_t launch_terms_combine(const double *out, double *hh, const double *dd, double cterm,
                                int64_t B, double *dh, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_terms_combine, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, out, hh,
                     dd, cterm, B, dh);
  return hipGetLastError();
}

// Time-domain SNRs from the two inner products (Sec. II.B item 7): the matched-filter
// rho_mf = <d,h> / sqrt(<h,h>), the optimal rho_opt = sqrt(<h,h>) and the effective
// rho_eff^2 = <d,d> - <d-h,d-h>, which expands to 2 <d,h> - <h,h>.
__global__ void k_snr(const double *__restrict__ dh, const double *__restrict__ hh, int64_t B,
                      double *__restrict__ rho_mf, double *__restrict__ rho_opt,
                      double *__restrict__ rho_eff2) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const double a = dh[b], c = hh[b];
  const double r = sqrt(c);
  if (rho_mf) rho_mf[b] = a / r;
  if (rho_opt) rho_opt[b] = r;
  if (rho_eff2) rho_eff2[b] = 2.0 * a - c;
}

hipError_t launch_snr(const double *dh, const double *hh, int64_t B, double *rho_mf,
                      double *rho_opt, double *rho_eff2, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_snr, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, dh, hh, B, rho_mf,
                     rho_opt, rho_eff2);
  return hipGetLastError();
}

}  // namespace tda
