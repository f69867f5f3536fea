// Internal declarations shared by the libtda translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/tda.h"

namespace tda {

// Row padding unit and block size of the FP64 triangular solve (rows per block row).
constexpr int TB = 256;
// Panel width of the FP64 Cholesky.
constexpr int CP = 128;
// Columns (templates) per workgroup of the FP64 triangular solve.
constexpr int BC = 32;
// Mixed path: template padding unit (the transposed product covers 256 templates).
constexpr int MT = 256;

// ---------------------------------------------------------------- device-side work descriptors

// One (handle, data, templates) evaluation of the FP64 solve.
struct TrsmItem {
  const double *panels;     // packed panels (see pack_panels)
  const int64_t *panel_off; // [nblk] element offset of each block row's panel
  const int32_t *blk_first; // [nblk] first block row of the segment containing the block row
  const int32_t *idx;       // [n_pad] sample index of each padded row, -1 = padding
  const double *d;          // data (MODE_LOGLIK)
  const double *H;          // templates, row stride ldh (MODE_LOGLIK)
  int64_t ldh;
  const double *const *Hrows; // optional per-template row pointers (overrides H, ldh)
  double *out;              // [B] results (MODE_LOGLIK)
  double *scratch;          // solution rows of every column tile of this item
  double cterm;             // -1/2 logdet - N_eff/2 log 2 pi
  int32_t B;                // templates (MODE_LOGLIK) or columns (MODE_IDENTITY)
  int32_t mode;
};

enum { MODE_LOGLIK = 0, MODE_IDENTITY = 1 };

// Explicit-inverse FP64 evaluation (the paper's CDO form, Sec. III.A.2): w = W (d - h)
// with W = L^-1 held in FP64 in compact column tiles (tile ct of 32 columns holds rows
// [rb[ct], segment end) at w64[off[ct] + (r - rb[ct]) 32 + c % 32]) and the residuals
// packed per template, R[b][r] = d[idx[r]] - h_b[idx[r]] (0 at padding), row stride n_pad.
// A workgroup forms a 256-row block of w for 64 templates and writes per template the
// sum of squares of its rows to part[block][b]; cdo_finish sums the blocks in order.
constexpr int CDO_T = 64;  // templates per workgroup
struct CdoItem {
  const double *w64;
  const int64_t *w64_off;  // [n_pad / 32]
  const int32_t *w64_rb;   // [n_pad / 32]
  const int32_t *blk_first, *blk_last;
  const int32_t *idx;      // [n_pad]
  const double *d;
  const double *H;
  int64_t ldh;
  double *R;               // [Bp][n_pad]
  double *part;            // [nblk][Bp]
  double *out;             // [B]
  double cterm;
  int32_t B, Bp, nblk, n_pad;
};
hipError_t launch_cdo_pack(const CdoItem *it_dev, const CdoItem &it, hipStream_t s);
hipError_t launch_cdo(const CdoItem *it_dev, const int4 *work, int64_t n_work, hipStream_t s);
hipError_t launch_cdo_finish(const CdoItem *it_dev, int64_t B, hipStream_t s);

// One workgroup of the FP64 solve: 32 columns of one item over block rows [blk_begin, blk_end).
struct TrsmTile {
  int32_t item;
  int32_t c0;
  int32_t blk_begin;
  int32_t blk_end;
  int64_t w_off;  // offset (doubles) of this tile's rows in item.scratch; row r at (r - blk_begin*TB)*BC
};

// Mixed path, per item.
struct MixItem {
  // whitening operator copies (BF16 hi/lo, fragment layouts)
  const uint16_t *wa_hi, *wa_lo;   // W, row blocks, lower part
  const uint16_t *wb_hi, *wb_lo;   // W^T, column blocks
  const int64_t *wa_off, *wb_off;  // [nblk] element offsets
  const int32_t *blk_first;        // [nblk]
  const int32_t *blk_last;         // [nblk] last block row of the segment (inclusive)
  const int32_t *idx;              // [n_pad]
  // operands / results
  const double *H;
  int64_t ldh;
  const double *const *Hrows;      // optional per-template row pointers
  uint16_t *hs_hi, *hs_lo;         // split templates, fragment layout, [Bp/32][tks][64][8]
                                   // (another item's, when hs_shared)
  uint16_t *es_hi, *es_lo;         // split residual e, same layout (this item's own buffer),
                                   // written by the refinement
  uint16_t *w0_hi, *w0_lo;         // split W h, same layout as hs
  int64_t tks;                     // k-steps per template tile in those layouts (n_pad/16 + TKS_PAD)
  float *y0;                       // [Bp][n_pad]
  double *e64;                     // [Bp][n_pad] FP64 scratch of the split refinements (or null)
  double *corr_part;               // [nblk][Bp] per-block sums of (W e)^2
  double *qpart;                   // [Bp] FP64 part of the quadratic form
  double *out;
  double *hh_out;                  // optional [B]: h^T C^-1 h (refined part added here)
  double cterm;
  int32_t B, Bp;                   // templates, padded to a multiple of MT
  int32_t nblk;
  int32_t n_pad;
  int32_t hs_shared;               // hs is split by an earlier item (same templates and rows)
  int32_t pad0;
};

// Template tiles of the split layouts are n_pad/16 + TKS_PAD fragments apart: without the
// pad the tiles sit a power of two apart (1 MB at N = 16384) and the tiles read together
// by the products would fall on the same memory channels.
constexpr int64_t TKS_PAD = 5;

// Refinement (FP64 FFT Toeplitz quadratic form), per item.
struct SegDev {
  int64_t offset, length;  // sample range of the segment
  int64_t row0;            // first padded row
  int64_t nkeep;           // retained rows of the segment
  int64_t npad;            // padded rows of the segment
  int64_t m;               // circulant length (power of two >= 2 length)
  int32_t log2m;
  int32_t pad0;
  const double *lam;       // [m] circulant eigenvalues
  const double *tw;        // [2m] cos/sin of 2 pi r / m
  const double *ptw;       // [2 rl_tw_size(log2m - 2)] pass twiddles of the m/4-point DFT
};

// In-LDS refinement: the m/4-point complex DFTs (h = m/4 <= 2^RL_LHMAX) run in one
// workgroup's LDS as in-place Stockham passes of radix 2^L (L <= 4).  The pass plan for
// h = 2^LH: ceil(LH / 4) passes of near-equal radix, larger radices first.
constexpr int RL_LHMAX = 13;
constexpr int64_t RL_MAX_M = (int64_t)4 << RL_LHMAX;
// Twice that length still refines in LDS, with each m/4-point DFT split into two halves;
// four times, into quarters, three of which wait in per-workgroup global scratch of
// RL_QUAD_SCRATCH complex doubles (launches with such segments run RL_QUAD_WG workgroups).
constexpr int64_t RL_MAX_M_SPLIT = 2 * RL_MAX_M;
constexpr int64_t RL_MAX_M_QUAD = 4 * RL_MAX_M;
constexpr int64_t RL_QUAD_SCRATCH = (int64_t)3 << RL_LHMAX;
constexpr int RL_QUAD_WG = 512;
__host__ __device__ constexpr int rl_npass(int LH) { return LH <= 4 ? 1 : (LH + 3) / 4; }
__host__ __device__ constexpr int rl_L(int LH, int p) {
  return LH / rl_npass(LH) + (p < LH % rl_npass(LH) ? 1 : 0);
}
// log2 of the sub-transform length entering pass p
__host__ __device__ constexpr int rl_lns(int LH, int p) { return p == 0 ? 0 : rl_lns(LH, p - 1) + rl_L(LH, p - 1); }
// offset of pass p's twiddles w_{Ns R}^{q k} (k < Ns, q = 1 .. R-1, stored [k][q-1])
__host__ __device__ constexpr int rl_off(int LH, int p) {
  return p <= 1 ? 0 : rl_off(LH, p - 1) + (((1 << rl_L(LH, p - 1)) - 1) << rl_lns(LH, p - 1));
}
__host__ __device__ constexpr int rl_tw_size(int LH) { return rl_off(LH, rl_npass(LH)); }

struct RefItem {
  const SegDev *segs;
  int32_t n_segs;
  int32_t B;
  const int32_t *pos2row;  // [N] padded row of each sample, -1 = excluded
  const float *y0;         // [Bp][n_pad]
  const double *H;
  int64_t ldh;
  const double *const *Hrows;
  const double *yd_pos;    // [N] C^-1 d scattered to sample positions (0 at excluded)
  const double *qdd;       // scalar: this call's q_dd (DataCheck::qdd)
  const int32_t *idx;      // [n_pad] sample index of each padded row, -1 = padding
  double *e64;             // [Bp][n_pad] FP64 scratch of the split refinements (else null)
  uint16_t *es_hi, *es_lo; // residual e output, split (BF16 hi/lo) in the fragment layout
  int64_t tks;             // k-steps per template tile in that layout
  double *qpart;           // [Bp] FP64 part of q output
  double *out;
  double *dh_out;          // optional [B]: d^T C^-1 h
  double *hh_out;          // optional [B]: the refined h^T C^-1 h before the correction
  double cterm;
  int32_t n_pad;
  int32_t pad0;
};

// Row b of the templates of an item (explicit row table, or base + b * ldh).
template <class Item>
__device__ __forceinline__ const double *template_row(const Item &it, int64_t b) {
  return it.Hrows ? it.Hrows[b] : it.H + b * it.ldh;
}

// ---------------------------------------------------------------- kernel timing
// When enabled, timed_begin/timed_end bracket a launch with events on its stream.
struct TimedScope {
  const char *name;
  hipStream_t stream;
  int slot;
  TimedScope(const char *n, hipStream_t s);
  ~TimedScope();
};

// ---------------------------------------------------------------- launchers (kernels_*.hip)

hipError_t launch_assemble(const double *acf, const int32_t *idx, int64_t n_keep, int64_t n_pad,
                           double *A, hipStream_t s);
hipError_t launch_cholesky(double *A, int64_t n, double *dinv, double *logdiag, int32_t *fail,
                           hipStream_t s);
hipError_t launch_diag_inverse(const double *A, int64_t n, const double *dinv128, double *dinv256,
                               hipStream_t s);
hipError_t launch_pack_panels(const double *A, int64_t n, int64_t row0, const double *dinv256,
                              double *panels, const int64_t *panel_off_host, int32_t blk0,
                              int32_t nblk_seg, hipStream_t s);
hipError_t launch_sum_logdet(const double *logdiag, int64_t count, double *logdet, hipStream_t s);
hipError_t launch_trsm_f64(const TrsmItem *items, const TrsmTile *tiles, int64_t n_tiles,
                           hipStream_t s);
hipError_t launch_trsm_f64_single(const TrsmItem &it, int32_t nblk, int64_t n_tiles,
                                  hipStream_t s);
hipError_t launch_combine(const double *parts, const int64_t *part_off, const int32_t *group_of,
                          int64_t n_items, double *const *outs, const int64_t *Bs,
                          int64_t n_groups, int64_t max_B, hipStream_t s);
void register_kernel_attributes();
hipError_t launch_scatter(const int64_t *desc, int64_t n, const double *src, hipStream_t s);
// <h,h> = -2 (hh - cterm) in place and, if dh != NULL, <d,h> = out - dd[0] + <h,h>/2
// Whitened residuals out of the single-item FP64 solve's scratch (column tile t holds
// row r of its 32 templates at scratch[(t n_pad + r) 32 + c]): wres[b][retpos[r]] for the
// retained rows (retpos >= 0), row stride ldw.
hipError_t launch_whiten_export(const double *scratch, const int32_t *retpos, int64_t n_pad,
                                int64_t B, double *wres, int64_t ldw, hipStream_t s);
// rho_mf = dh / sqrt(hh), rho_opt = sqrt(hh), rho_eff^2 = 2 dh - hh (NULL outputs skipped)
hipError_t launch_snr(const double *dh, const double *hh, int64_t B, double *rho_mf,
                      double *rho_opt, double *rho_eff2, hipStream_t s);
hipError_t launch_terms_combine(const double *out, double *hh, const double *dd, double cterm,
                                int64_t B, double *dh, hipStream_t s);

// mixed
hipError_t launch_split_w(const double *w64, const int64_t *w64_off, const int32_t *w64_rb,
                          const int32_t *blk_first, const int32_t *blk_last, int32_t nblk,
                          uint16_t *wa_hi, uint16_t *wa_lo, const int64_t *wa_off,
                          uint16_t *wb_hi, uint16_t *wb_lo, const int64_t *wb_off,
                          int64_t max_k, int64_t unused, hipStream_t s);
// Whitened-data cache of a mixed handle (device): fingerprint of the retained samples of
// the data it was computed from, valid flag, and q_dd = dbar^T dbar.
struct DataCache {
  uint64_t fp;
  uint64_t valid;
  double qdd;
  double pad;
};
// Per call and handle (device, in the call's workspace): the data's fingerprint, whether
// the whitening kernels run, and the q_dd the refinement uses (NaN: data the handle can
// no longer whiten).  qdd is the first member: RefItem::qdd points at it.
struct DataCheck {
  double qdd;
  uint64_t fp;
  int32_t stale;
  int32_t pad[3];
};
hipError_t launch_data_check(const double *d, const int32_t *idx, int32_t n_pad, DataCache *cache,
                             DataCheck *chk, int32_t can_whiten, int32_t force, hipStream_t s);
// dbar, y_d, y_d at sample positions and q_dd, when chk->stale; publishes the fingerprint
hipError_t launch_data_whiten(const double *w64, const int64_t *w64_off, const int32_t *w64_rb,
                              const int32_t *blk_first, const int32_t *blk_last, const int32_t *idx,
                              const int32_t *pos2row, int32_t n_pad, int64_t N, const double *d,
                              double *dbar, double *yd, double *yd_pos, DataCache *cache,
                              DataCheck *chk, hipStream_t s);
hipError_t launch_lambda(const double *acf, int64_t length, int64_t m, double *tw, double *lam,
                         double *ptw, hipStream_t s);
// Split the gathered templates h into the fragment layout of the products: one launch over
// all items; max_chunks = max over items of (Bp/32)(n_pad/16) 64
hipError_t launch_split_h(const MixItem *items, int32_t n_items, int64_t max_chunks,
                          hipStream_t s);
hipError_t launch_corr(const MixItem *items, const int4 *work, int64_t n_work, int variant,
                       hipStream_t s);
hipError_t launch_finish(const MixItem *items, const int2 *work, int64_t n_work, hipStream_t s);
// fwd/corr entries: (item, row block, group of 128 templates, 0);
// bwd entries: (item, column block, group of 256 templates, half of the block)
// variant: 1 or 2 waves per SIMD (chosen per shape by the autotuner)
hipError_t launch_trmm_fwd(const MixItem *items, const int4 *work, int64_t n_work, int variant,
                           hipStream_t s);
hipError_t launch_trmm_bwd(const MixItem *items, const int4 *work, int64_t n_work, int variant,
                           hipStream_t s);

// ---------------------------------------------------------------- autotuner (autotune.hip)
// Chooses, per (kernel, row bucket, template bucket), the fastest variant among
// `variants` on the caller's stream the first time the key is seen (that call
// synchronises): one untimed launch of each, then three timed rounds over all of them,
// and the smallest median wins.  Choices persist in-process and, when the
// environment variable TDA_AUTOTUNE_CACHE names a file, across processes (text lines
// "kernel rows_log2 templates_log2 variant").  TDA_AUTOTUNE=0 disables timing and uses
// the first variant.
int autotune_pick(const char *kernel, int64_t rows, int64_t templates, const int *variants,
                  int n_variants, hipStream_t s, hipError_t (*launch)(void *ctx, int variant),
                  void *ctx);
void register_mixed_attributes();
// work entries (item, template a, template b or -1, 0): two templates share one DFT
hipError_t launch_refine(const RefItem *items, const int4 *work, int64_t n_work, double *scratch,
                         int64_t scratch_per_wg, int32_t n_wg, hipStream_t s);
// Gohberg-Semencul evaluation (segments without excluded samples, m <= RL_MAX_M).
struct GsSeg {
  int64_t offset, length;  // sample range of the segment (all samples retained)
  int64_t m;               // circulant length (power of two >= 2 length)
  int32_t log2m;
  int32_t pad0;
  double inv_x0;           // 1 / (C^-1)_00
  const double *tw;        // [2m] cos/sin of 2 pi r / m
  const double *ptw;       // pass twiddles of the m/4-point DFT
  const double *M1, *M2;   // [2m] conj(DFT_m) of x = C^-1 e_1 and of (0, x_{n-1}, ..., x_1)
};

struct GsItem {
  const GsSeg *segs;
  int32_t n_segs;
  int32_t B;
  const double *d;                 // [N] data
  const double *H;                 // templates, rows of stride ldh
  int64_t ldh;
  const double *const *Hrows;      // optional per-template row pointers
  double *out;                     // [B] -q/2 + cterm
  double cterm;
};

__device__ __forceinline__ const double *gs_template_row(const GsItem &it, int64_t b) {
  return it.Hrows ? it.Hrows[b] : it.H + b * it.ldh;
}

// Levinson-Durbin for the first column of the inverse of the symmetric Toeplitz matrix
// with first column acf[0..n): x = C^-1 e_1, log det C = sum log E_k; *fail = first k with
// E_k <= 0 or not finite (else -1).  One workgroup; n <= GS_MAX_LEN, with the
// coefficients in LDS up to RL_MAX_LEV and in x (global memory) beyond.
constexpr int RL_MAX_LEV = 16384;
// Longest Gohberg-Semencul segment: its circulant (m >= 2 n) runs through the in-LDS
// transforms split in quarters.
constexpr int GS_MAX_LEN = (int)(RL_MAX_M_QUAD / 2);
hipError_t launch_levinson(const double *acf, int64_t n, double *x, double *logdet,
                           int32_t *fail, hipStream_t s);
// conj(DFT_m) of x zero-padded and of (0, x_{n-1}, ..., x_1) zero-padded
hipError_t launch_gs_spectra(const double *x, int64_t n, int64_t m, const double *tw,
                             double *M1, double *M2, hipStream_t s);
// q_b over the segments of each item, out[b] = -q_b/2 + cterm; work entries (item, b).
// Workgroup g uses scratch + g scratch_stride doubles: the parked even part, and from qoff
// (even; -1 = none) RL_QUAD_SCRATCH complex doubles for segments with m > RL_MAX_M_SPLIT.
hipError_t launch_gs(const GsItem *items, const int2 *work, int64_t n_work, double *scratch,
                     int64_t scratch_stride, int64_t qoff, int32_t n_wg, hipStream_t s);

// In-LDS refinement for launches whose segments all have m <= RL_MAX_M_QUAD; work entries
// (item, template).  qscratch: RL_QUAD_WG x RL_QUAD_SCRATCH complex doubles when a segment
// has m > RL_MAX_M_SPLIT, else NULL.
hipError_t launch_refine_lds(const RefItem *items, const int2 *work, int64_t n_work,
                             double *qscratch, hipStream_t s);

// ---------------------------------------------------------------- internal entry points (tda_api.hip)
struct MultiCtx;
MultiCtx *multi_ctx_create();
void multi_ctx_destroy(MultiCtx *mc);
// Batched evaluation with a private workspace; hrows (optional) gives per-item device
// arrays of template row pointers.  Caller serialises use of one MultiCtx.
tda_status multi_eval(MultiCtx *mc, const tda_work *items, const double *const *const *hrows,
                      int64_t n_items, int32_t precision, hipStream_t s);
int handle_device(tda_handle h);
int64_t handle_n(tda_handle h);
size_t handle_bytes(tda_handle h);
// Device workspace a batched evaluation takes: per item of B templates (the template and
// residual splits, y0 and e for the mixed path, the solve scratch for FP64), plus a part
// shared by the launch (the FFT scratch of its longest circulant, the largest over items);
// 0 where the precision keeps none worth counting.
size_t item_ws_bytes(tda_handle h, int64_t B, int32_t precision);
size_t launch_ws_fixed_bytes(tda_handle h, int32_t precision);
// bytes a private batched-evaluation context holds now
size_t multi_ctx_held(MultiCtx *mc);
bool handle_ready(tda_handle h, int32_t precision);
tda_status handle_set_data(tda_handle h, const double *d, hipStream_t s);
tda_status set_error(tda_status st, const char *msg);
void register_acf_attributes();

}  // namespace tda
