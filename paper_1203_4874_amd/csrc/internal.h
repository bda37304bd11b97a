// Internal launch interface between the C ABI (api.hip) and the kernel
// translation units.  Not part of the public ABI.
//
// Every kernel works on "work items" of one queue (a phase of the path).  A
// launch covers the frames of a call (one or many): their descriptors and
// per-queue item prefix sums sit in device memory (the workspace head); the
// grid may be smaller than the item count, each workgroup then looping over
// items (a persistent launch), and finds each item's frame by binary search.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

#include "cbp.h"
#include "common.h"
#include "fft_core.h"

namespace cbp {

// Work queues, one per kernel.
enum queue_id {
  Q_DIAG = 0, Q_FOLD, Q_EVAL_COLS, Q_EVAL_ROWS, Q_ROW_FWD, Q_GRAM, Q_GRAMM, Q_SAMPLE, Q_FINALIZE, Q_COL,
  Q_ROW_INV, Q_TWID, Q_SIZE_PROBE, Q_KRDFT, Q_COUNT
};

// Frames per batched launch (the item prefix sums of one launch sit in LDS).
constexpr int BATCH_CHUNK = 256;

// Geometry and workspace offsets of one frame (host side; offsets in bytes
// from the frame's workspace base).
struct frame_plan {
  int H1, W1, H2, W2, Hmax, Wmax;
  int m, n, k1, k2, S, N;  // N = k1 + k2
  int nch;
  int rpg, RG;             // fold row-group size (multiple of S) and count
  int Py, Px, hx;          // FFT grid and half-spectrum width
  int hxp;                 // row pitch of T and U (entries): hx rounded up to 128 bytes
  int cw;                  // columns per workgroup in the column pass
  fft_plan fy, fx;
  int twy, twx;            // column pass: col_table_entries; row passes: the row plan's pass tables
  size_t off_fpart, off_ex, off_ey, off_corr, off_xvec, off_pq, off_kern,
      off_t1, off_t2, off_u, off_feat, off_wts, off_kalt, off_twxd, off_kr, total;
};

// Everything a kernel needs about one frame (device pointers).
struct frame_desc {
  const void* b1;
  const void* b2;
  int64_t p1, p2;    // row pitch (elements)
  int64_t cs1, cs2;  // channel stride (elements; 0 for one channel)
  int H1, W1, H2, W2, Hmax, Wmax, nch;
  int ncf;           // evaluated (channel, frame) slots: 2 nch (1 for the one-frame evaluation entry point)
  int m, n, k1, k2, S, N;
  int rpg, RG, Py, Px, hx, cw;
  fft_plan fy, fx;
  // workspace regions
  double* fpart;
  c64* ex;
  c64* ey;
  cdd* corr;
  c64* xvec;
  c64* pq;
  void* t1;
  void* t2;
  void* u;
  // outputs
  double* K1;
  double* K2;
  void* out;
  int64_t opitch, ocs;
  double lambda;
  cbp_diag* diag;
  // learned form (NULL otherwise): per-sample features [2S][32] (written by
  // the eigen-solves) and the network's weights [2S] + tau (read by the
  // assembly)
  float* feat;
  double* wts;
  double* Kalt;   // the plain method's kernels (fallback of the learned form), 2 x CBP_MAX_K^2
  // twiddle table exp(-2 pi i t / Px), FP64 (the kernels' row DFTs in the
  // column pass; the FFT passes build short tables of their own in LDS)
  c64* twxd;
  // paper-faithful variants (CBP_FLAG_DIVIDE_B1 / SCALE_K1 / ONE_AXIS as
  // VAR_* bits; 0 = the default method) and VAR_FP64_GRAM
  int variant;
  int hxp;           // row pitch of T and U (entries), a multiple of 128 bytes
  // the kernels' row DFTs at every half-spectrum column, [hx][2][CBP_MAX_K]
  // (transform type), for the column pass
  void* kr;
};
constexpr int VAR_DIVIDE_B1 = 1, VAR_SCALE_K1 = 2, VAR_ONE_AXIS = 4;
// The Gram is formed on the matrix cores (MFMA64, MFMA32, BF16): these forms
// work to the mixed-precision accuracy (kernels within 1e-3 of the FP64
// method), so the eigen-solves stop at the inverse-iteration vector (on the
// 1080p RGB stream within 2e-6 of the FP64 method's kernels; the
// double-double Newton refinement would take it to 3e-7, the level the FP64
// Gram's own rounding leaves, at a third of the solves' time).
constexpr int VAR_FP64_GRAM = 8;
__host__ __device__ inline int solve_refine_max(int variant) { return (variant & VAR_FP64_GRAM) ? 0 : 4; }

// Work items of each queue for one frame (the grid of a one-frame launch).
inline int queue_items(int q, const frame_plan& p) {
  const int ncf = 2 * p.nch;
  switch (q) {
    case Q_DIAG: return 1;
    case Q_FOLD: return ((p.Wmax + 63) / 64) * p.S * p.RG * ncf;
    case Q_EVAL_COLS: return ((p.Wmax + 15) / 16) * ncf;
    case Q_EVAL_ROWS: return ((p.Hmax + 1) / 2) * ncf;
    case Q_ROW_FWD: return p.nch * p.RG * p.S;   // (channel, row group, residue); rows y < Hmax of each
    case Q_GRAM: return (2 * p.N - 1) * p.S * 2;
    case Q_GRAMM: return p.S * 2;
    case Q_SAMPLE: return p.S * 2;
    case Q_FINALIZE: return 1;
    case Q_COL: return ((p.hx + p.cw - 1) / p.cw) * p.nch;
    case Q_ROW_INV: return ((p.m + 1) / 2) * p.nch;
    case Q_TWID: return (p.Px + 255) / 256;
    case Q_SIZE_PROBE: return 0;   // set by the size-estimation entry point (candidates x 2S)
    case Q_KRDFT: return (p.hx * 2 * CBP_MAX_K + 255) / 256;
  }
  return 0;
}

// The frames of a launch as the kernels see them (device memory).
struct batch_ref {
  const frame_desc* descs;  // nframes descriptors
  const int* starts;        // [Q_COUNT][nframes + 1] item prefix sums
  int nframes;
  int* ctr;                 // [CTR_COUNT] item counters of the dynamic launches (zeroed by the first launch)
};

// Item counters of a chunk's dynamically scheduled launches, eight each (one
// per XCD): the row pass, the inverse rows, and the column pass per filter
// group (4, 2, 1).
constexpr int CTR_ROW_FWD = 0, CTR_ROW_INV = 8, CTR_COL = 16, CTR_COUNT = 64;
static_assert(CTR_COL + 3 * 8 <= CTR_COUNT, "counter block");

// Rows per group of the column filter's kernel-spectrum evaluation (rows
// y + j N/g, j < g, share one Horner chain in w_N^(g y)): 4, 2 or 1 as N
// allows.
__host__ __device__ inline int col_group_size(int N) { return (N & 3) == 0 ? 4 : (N & 1) == 0 ? 2 : 1; }

// Column-pass twiddle entries beyond the full table: the filter's
// w_N^(g y), y < N / g (g = col_group_size(N) > 1), and the pass tables of
// plan p.
inline int col_table_entries(const fft_plan& p) {
  const int g = col_group_size(p.N);
  return (g > 1 ? p.N / g : 0) + pass_table_entries(p);
}

#if defined(__HIPCC__)
// Items [first, end) step `step` of this workgroup.  Workgroups are
// dispatched to the 8 XCDs round robin (workgroup b on XCD b mod 8); with a
// grid that is a multiple of 8, XCD x takes the contiguous item range
// [x T / 8, (x + 1) T / 8), so neighbouring items (the lags of one sample,
// adjacent rows and strips of one frame) share their inputs in one XCD's L2.
__device__ inline void xcd_items(int T, int b, int G, int& first, int& end, int& step) {
  if (G < 8 || (G & 7) != 0) {
    first = b;
    end = T;
    step = G;
    return;
  }
  const int x = b & 7;
  first = (int)(((int64_t)x * T) >> 3) + (b >> 3);
  end = (int)(((int64_t)(x + 1) * T) >> 3);
  step = G >> 3;
}

// Items [0, T) of a persistent grid handed out dynamically: workgroup b of G
// takes the items of its XCD's range [x T / 8, (x + 1) T / 8) (x = b mod 8,
// the XCD it runs on when G is a multiple of 8; otherwise one range) one at
// a time from that range's counter, so a workgroup that starts late (its CU
// still busy with another launch) takes fewer items instead of delaying the
// launch, and adjacent items still share an XCD's L2.
struct dyn_items {
  int* ctr;
  int lo, hi;
  // one thread: the next item, hi when the range is exhausted
  __device__ int take() const {
    const int i = lo + atomicAdd(ctr, 1);
    return i < hi ? i : hi;
  }
};
__device__ inline dyn_items make_dyn_items(int* ctr8, int T, int b, int G) {
  if (G < 8 || (G & 7) != 0) return dyn_items{ctr8, 0, T};
  const int x = b & 7;
  return dyn_items{ctr8 + x, (int)(((int64_t)x * T) >> 3), (int)(((int64_t)(x + 1) * T) >> 3)};
}

// Run body(frame, item) for every item of queue Q owned by workgroup b of
// the G workgroups serving Q (a launch may split its workgroups between
// queues).  The body may use __syncthreads(); a barrier separates
// consecutive items.
template <int Q, typename F>
__device__ inline void for_items_part(const batch_ref& br, int b, int G, F&& body) {
  __shared__ int st[BATCH_CHUNK + 1];
  const int nf = br.nframes;
  const int* s = br.starts + (size_t)Q * (nf + 1);
  for (int t = threadIdx.x; t <= nf; t += blockDim.x) st[t] = s[t];
  __syncthreads();
  int first, end, step;
  xcd_items(__builtin_amdgcn_readfirstlane(st[nf]), b, G, first, end, step);
  // descriptors are read-only while kernels run: reading them through the
  // constant address space with a wave-uniform index lets the scalar unit
  // load them into SGPRs
  for (int it = first; it < end; it += step) {
    int lo = 0, hi = nf;  // st[lo] <= it < st[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (st[mid] <= it) lo = mid;
      else hi = mid;
    }
    const int fi = __builtin_amdgcn_readfirstlane(lo);
    const int base = __builtin_amdgcn_readfirstlane(st[fi]);
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) frame_desc cdesc;
    const frame_desc d = ((const cdesc*)br.descs)[fi];
#else
    const frame_desc d = br.descs[fi];
#endif
    body(d, it - base);
    __syncthreads();
  }
}

// Every item of queue Q owned by this workgroup of the whole launch.
template <int Q, typename F>
__device__ inline void for_items(const batch_ref& br, F&& body) {
  for_items_part<Q>(br, (int)blockIdx.x, (int)gridDim.x, body);
}

// w_t = exp(-2 pi i t / S), t < S, into tw (the workgroup's threads).
__device__ inline void unit_twiddles(c64* tw, int S) {
  for (int t = threadIdx.x; t < S; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)S, &s, &c);
    tw[t] = {c, s};
  }
}

// sum_i p[(x0 + i step) stride] over x0 + i step < W, in increasing i, in
// FP64: eight loads are issued before their (ordered) additions.
template <typename T>
__device__ __attribute__((always_inline)) inline double fold_strided(const T* p, int stride, int x0, int step, int W) {
  double acc = 0.0;
  int x = x0;
  for (; x + 7 * step < W; x += 8 * step) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(x + u * step) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (double)v[u];
  }
  for (; x < W; x += step) acc += (double)p[(size_t)x * stride];
  return acc;
}

// sum_r f[r fs] w_(j r mod S), r < S, in increasing r (w from
// unit_twiddles): four terms' operands are loaded before their (ordered)
// accumulation.
__device__ __attribute__((always_inline)) inline c64 dft_at(const double* f, int fs, const c64* tw, int S, int j) {
  c64 e = {0.0, 0.0};
  int t = 0, r = 0;
  for (; r + 4 <= S; r += 4) {
    double fv[4];
    c64 wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      fv[u] = f[(r + u) * fs];
      wv[u] = tw[t];
      t += j;
      if (t >= S) t -= S;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      e.re += fv[u] * wv[u].re;
      e.im += fv[u] * wv[u].im;
    }
  }
  for (; r < S; ++r) {
    e.re += f[r * fs] * tw[t].re;
    e.im += f[r * fs] * tw[t].im;
    t += j;
    if (t >= S) t -= S;
  }
  return e;
}

// One item of the column evaluation (Sec. 4 eq. 3: the S-point DFT of the
// column fold): the row-group partials of 16 columns of one (channel, frame)
// summed in group order into F[r][column], then EX[cf][j][x] = sum_r
// w_j^r F[r][x].  256 threads: 16 columns x 16 residues / frequencies in
// flight, each thread two residues when S > 16.  F (CBP_MAX_S x 16 doubles) and tw (CBP_MAX_S) are LDS scratch.
// Items: (column block, cf).
static_assert(CBP_MAX_S <= 32, "the column evaluation holds residues ty and ty + 16 per thread");
__device__ inline void eval_cols_item(const frame_desc& d, int item, double (*F)[16], c64* tw) {
  const int nx = (d.Wmax + 15) / 16;
  const int bx = item % nx, cf = item / nx;
  const int S = d.S, Wmax = d.Wmax, RG = d.RG;
  const int W = (cf & 1) ? d.W2 : d.W1;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int x = bx * 16 + tx;
  unit_twiddles(tw, S);
  // residues ty and ty + 16 (S <= 32) at once: eight groups' loads of each in
  // flight; even groups into s0, odd into s1, in group order
  {
    const bool h0 = ty < S && x < W, h1 = ty + 16 < S && x < W;
    const size_t gs = (size_t)d.ncf * S * Wmax;
    const double* p0 = d.fpart + ((size_t)cf * S + ty) * Wmax + x;
    const double* p1 = p0 + (size_t)16 * Wmax;
    double s0 = 0.0, s1 = 0.0, t0 = 0.0, t1 = 0.0;
    int g = 0;
    for (; g + 8 <= RG; g += 8) {
      double v[8], w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = h0 ? p0[(size_t)(g + u) * gs] : 0.0;
        w[u] = h1 ? p1[(size_t)(g + u) * gs] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        s0 += v[u];
        s1 += v[u + 1];
        t0 += w[u];
        t1 += w[u + 1];
      }
    }
    for (; g + 2 <= RG; g += 2) {
      if (h0) {
        s0 += p0[(size_t)g * gs];
        s1 += p0[(size_t)(g + 1) * gs];
      }
      if (h1) {
        t0 += p1[(size_t)g * gs];
        t1 += p1[(size_t)(g + 1) * gs];
      }
    }
    if (g < RG) {
      if (h0) s0 += p0[(size_t)g * gs];
      if (h1) t0 += p1[(size_t)g * gs];
    }
    if (ty < S) F[ty][tx] = s0 + s1;
    if (ty + 16 < S) F[ty + 16][tx] = t0 + t1;
  }
  __syncthreads();
  if (x >= W) return;
  for (int j = ty; j < S; j += 16) d.ex[((size_t)cf * S + j) * Wmax + x] = dft_at(&F[0][tx], 16, tw, S, j);
}
#endif

// ---------------------------------------------------------------- phase timing
// Phases of one call, in launch order (also the names cbp_profile_phase_name
// returns).
enum phase_id {
  PH_FOLD = 0, PH_EVAL_COLS, PH_EVAL_ROWS, PH_GRAM, PH_SAMPLE, PH_FINALIZE,
  PH_ROW_FWD, PH_COL_FILTER, PH_ROW_INV, PH_KR_DFT, PH_COUNT
};
// Record the start / end of a phase on a stream when timing is enabled
// (no-ops otherwise).  Implemented in api.hip.
void prof_begin(int phase, hipStream_t st);
void prof_end(int phase, hipStream_t st);

// ---------------------------------------------------------------- launchers
// Each launches one queue over `grid` workgroups (any grid >= 1 covers every
// item; a multiple of 8 enables the XCD-aware item ranges).
// The head of a small one-chunk call (frame descriptors, then the per-queue
// item prefix sums of the chunk) passed by value to the first launch, which
// reads its descriptors from it and stores it into the workspace head for the
// launches that follow: no host-to-device copy precedes the call's kernels.
constexpr int kInlineHeadMax = 1664;   // three frames
struct inline_head {
  int ndesc_bytes;    // nframes * sizeof(frame_desc); 0: no inline head
  int nstart_bytes;   // Q_COUNT * (nframes + 1) * sizeof(int)
  int pad[2];
  alignas(16) char bytes[kInlineHeadMax];
};

// eval.hip.  launch_fold runs the column fold on `grid` workgroups and, on
// twid_grid more, the twiddle tables of every frame (items of Q_TWID; the
// FFT passes need them, the fold does not, so they share one launch).  With
// ih, the launch carries the call's head (br then points at its place in the
// workspace).
template <typename T>
hipError_t launch_fold(const batch_ref& br, int grid, int twid_grid, const inline_head* ih, hipStream_t st);
hipError_t launch_eval_cols(const batch_ref& br, int grid, hipStream_t st);
template <typename T>
hipError_t launch_eval_rows(const batch_ref& br, int grid, hipStream_t st);

// recover.hip
hipError_t launch_diag_init(const batch_ref& br, int grid, hipStream_t st);
hipError_t launch_gram(const batch_ref& br, int grid, hipStream_t st);
// dense Gram matrices (2 S N N complex FP64, [pass][sample][p][q]); items of Q_GRAMM
hipError_t launch_gram_expand(const batch_ref& br, int grid, double* out, hipStream_t st);
hipError_t launch_sample(const batch_ref& br, int grid, int maxN, hipStream_t st);
// lean: every frame's scale solve runs without refinement or diagnostics
// (its coupling block shares the solver's X region: less LDS)
hipError_t launch_finalize(const batch_ref& br, int grid, int maxS, int learned, int plain_only, bool lean,
                           hipStream_t st);
// the learned form's judge: keeps the plain kernels where their per-sample
// residual objective is smaller (items of Q_FINALIZE)
hipError_t launch_judge(const batch_ref& br, int grid, hipStream_t st);
size_t finalize_lds_bytes(int S, int learned, bool lean = false);
size_t sample_lds_bytes(int N);

// gram_mfma.hip: the per-sample Gram on the matrix cores (fmt 0: FP32
// operands, 1: bfloat16), N = k1 + k2 <= 32; maxStride = the largest Wmax /
// Hmax of the launched frames.
hipError_t launch_gram_mfma(const batch_ref& br, int grid, int fmt, int maxStride,
                            hipStream_t st);
size_t gram_mfma_lds_bytes(int maxStride, int fmt);
void set_gram_mfma_attrs();

// fft.hip.  The row pass also writes the column fold's partials (the
// k_fold_cols result, bit for bit) and, with with_ey, the row evaluation EY
// (the k_eval_rows result, bit for bit) from the rows it already holds.
template <typename T>
hipError_t launch_row_fwd(const batch_ref& br, int grid, int maxPx, int maxTw, int with_ey, hipStream_t st);
template <typename T>
// gmask: the filter groups g (bit g) of the batch's frames; one launch per
// group, each taking the items of its frames
hipError_t launch_col(const batch_ref& br, int grid, int maxPy, int maxcw, int maxTw, int gmask, hipStream_t st);
template <typename T>
hipError_t launch_kernel_dft(const batch_ref& br, int grid, hipStream_t st);
template <typename T>
hipError_t launch_row_inv(const batch_ref& br, int grid, int maxPx, int maxTw, hipStream_t st);
size_t row_lds_bytes(int N, int twn, int esize);   // twn: pass twiddle-table entries
int row_fwd_per_cu(size_t lds, int esize);
size_t col_lds_bytes(int N, int cw, int twn, int esize);
int col_max_strip_elems(int esize);   // largest cw * Py the column pass holds
int col_threads(int N, int cw, int esize);
int col_per_cu(int N, int cw, int twn, int g, int esize);   // resident column-pass workgroups per CU   // column-pass workgroup size for a strip
void set_recover_attrs();
void set_fft_attrs();

// sizes.hip: blind kernel-size estimation.  Candidates k1' (ascending) with
// k2' = k1' - d; the probe's items are (candidate, pass, sample) of the one
// frame of br, whose plan holds the largest trial sizes; ratios is
// [n][2][S] device scratch.
struct size_cands {
  int n;                 // candidate count (<= CBP_MAX_K)
  int d;                 // k1 - k2 = H1 - H2
  int k1[CBP_MAX_K];
};
hipError_t launch_size_probe(const batch_ref& br, int grid, const size_cands& c, int nmax, int NLmax, double* ratios,
                             hipStream_t st);
hipError_t launch_size_decide(const size_cands& c, int S, const double* ratios, cbp_size_result* out,
                              hipStream_t st);
size_t size_probe_lds_bytes(int nmax, int NLmax);
void set_size_attrs();

// encoder.hip: the encoder's kernel draws, the blur and the 8-bit streams.
hipError_t launch_draw_pairs(unsigned long long seed, long long frame0, int nframes, int k1, int k2, int S,
                             double* K1s, double* K2s, int* attempts, double* min_ratio, hipStream_t st);
size_t draw_pairs_lds_bytes(int k1, int k2);
void set_encoder_attrs();
template <typename T>
hipError_t launch_blur(const T* L, int64_t lp, int64_t lcs, int m, int n, int nch, const double* K1, int k1,
                       const double* K2, int k2, T* B1, int64_t p1, int64_t cs1, T* B2, int64_t p2, int64_t cs2,
                       hipStream_t st);
template <typename T>
hipError_t launch_quantize(const T* src, int64_t sp, int64_t scs, unsigned char* dst, int64_t dp, int64_t dcs, int H,
                           int W, int nch, int drop, hipStream_t st);
template <typename T>
hipError_t launch_dequantize(const unsigned char* src, int64_t sp, int64_t scs, T* dst, int64_t dp, int64_t dcs,
                             int H, int W, int nch, hipStream_t st);

// mlp.hip: the learned form's network on every frame of the launch
// (features -> weights and tau); blob is a device mlp_blob.
hipError_t launch_mlp_frames(const batch_ref& br, int grid, const void* blob,
                             hipStream_t st);

}  // namespace cbp
