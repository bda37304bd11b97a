// C ABI of the CBP library (declared in include/cbp.h): host-side validation,
// frame plans and workspace layout, the launch chains (one frame; a batch of
// frames through work-list launches; a batch captured as a HIP graph), the
// batch autotuner, and phase timing.
//
// Every status returned here comes from host-side checks made before the
// first HIP call of the entry point, so invalid arguments never reach a
// kernel.  Launch failures are reported as CBP_E_DEVICE.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "mlp.h"

namespace cbp {

namespace {

constexpr size_t kAlign = 256;

// Scratch of the allocation-free entry point (cbp_deblur_noalloc): the
// workspace of one call, one copy per device, held until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: host
// code uses only the address hipGetSymbolAddress returns on each device
// (dev_state::scratch).
constexpr size_t kScratchBytes = size_t(48) << 20;
__device__ __align__(256) char scratch[kScratchBytes];
constexpr size_t kLdsLimit = 160 * 1024;
constexpr int kComputeUnits = 256;
constexpr int32_t kKnownFlags =
    CBP_FLAG_GRAPH | CBP_FLAG_AUTOTUNE | CBP_FLAG_DIVIDE_B1 | CBP_FLAG_SCALE_K1 | CBP_FLAG_ONE_AXIS;

// The VAR_* bits of a call's variant flags.
int variant_bits(int32_t flags) {
  return ((flags & CBP_FLAG_DIVIDE_B1) ? VAR_DIVIDE_B1 : 0) | ((flags & CBP_FLAG_SCALE_K1) ? VAR_SCALE_K1 : 0) |
         ((flags & CBP_FLAG_ONE_AXIS) ? VAR_ONE_AXIS : 0);
}

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int smooth7(int n) {
  int v = n < 1 ? 1 : n;
  for (;; ++v) {
    int r = v;
    for (int p : {2, 3, 5, 7})
      while (r % p == 0) r /= p;
    if (r == 1) return v;
  }
}

// Region sizes from monotone bounds of the frame dimensions, so that a layout
// for any frame within (maxH, maxW, maxk, S, nch) fits the size that
// cbp_workspace_size() reports for those bounds.
struct region_sizes {
  size_t fpart, ex, ey, corr, xvec, pq, kern, t, u, feat, wts, kalt, twxd, kr;
};

// Row pitch of T and U: hx entries of 2 esize bytes rounded up to 128 bytes.
int pitch_of(int hx, int esize) {
  const int per = 128 / (2 * esize);
  return (hx + per - 1) / per * per;
}

region_sizes regions(int Hmax, int Wmax, int kmax, int S, int nch, int esize) {
  region_sizes r;
  const int Px = smooth7(Wmax);
  const size_t hx = pitch_of((int)((size_t)Px / 2 + 1), esize);
  const size_t ncf = 2 * (size_t)nch;
  r.fpart = ((size_t)(Hmax + 31) / 32 + 1) * ncf * S * (size_t)Wmax * sizeof(double);
  r.ex = ncf * S * (size_t)Wmax * sizeof(c64);
  r.ey = ncf * S * (size_t)Hmax * sizeof(c64);
  r.corr = 2 * (size_t)S * (4 * (size_t)kmax - 1) * sizeof(cdd);
  r.xvec = 2 * (size_t)S * 2 * kmax * sizeof(c64);
  r.pq = 4 * (size_t)S * S * sizeof(c64);
  r.kern = 2 * (size_t)CBP_MAX_K * CBP_MAX_K * sizeof(double);
  r.t = (size_t)nch * Hmax * hx * 2 * esize;
  r.u = (size_t)nch * Hmax * hx * 2 * esize;
  r.feat = 2 * (size_t)S * 32 * sizeof(float);
  r.wts = (2 * (size_t)S + 1) * sizeof(double);
  r.kalt = 2 * (size_t)CBP_MAX_K * CBP_MAX_K * sizeof(double);
  r.twxd = (size_t)Px * sizeof(c64);
  r.kr = ((size_t)Px / 2 + 1) * 2 * CBP_MAX_K * 2 * esize;
  return r;
}

size_t layout(frame_plan* fp, const region_sizes& r) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  fp->off_fpart = take(r.fpart);
  fp->off_ex = take(r.ex);
  fp->off_ey = take(r.ey);
  fp->off_corr = take(r.corr);
  fp->off_xvec = take(r.xvec);
  fp->off_pq = take(r.pq);
  fp->off_kern = take(r.kern);
  fp->off_t1 = take(r.t);
  fp->off_t2 = take(r.t);
  fp->off_u = take(r.u);
  fp->off_feat = take(r.feat);
  fp->off_wts = take(r.wts);
  fp->off_kalt = take(r.kalt);
  fp->off_twxd = take(r.twxd);
  fp->off_kr = take(r.kr);
  fp->total = o;
  return o;
}

// a one-frame head always fits the first launch's arguments
static_assert(sizeof(frame_desc) % 16 == 0 &&
                  sizeof(frame_desc) + ((Q_COUNT * 2 * sizeof(int) + 15) & ~(size_t)15) <= kInlineHeadMax,
              "one frame's head must travel inline");

int nchunks(int nframes) { return (nframes + BATCH_CHUNK - 1) / BATCH_CHUNK; }

// Workspace head: the frame descriptors, the per-queue item prefix sums and
// the item counters of the dynamic launches of a batched call (frames follow
// it).
size_t head_desc_bytes(int nframes) { return align_up((size_t)nframes * sizeof(frame_desc)); }
size_t head_starts_bytes(int nframes) {
  return align_up((size_t)nchunks(nframes) * Q_COUNT * (BATCH_CHUNK + 1) * sizeof(int));
}
size_t head_bytes(int nframes) {
  return head_desc_bytes(nframes) + head_starts_bytes(nframes) +
         align_up((size_t)nchunks(nframes) * CTR_COUNT * sizeof(int));
}

int max_fft(int esize) { return esize == 4 ? CBP_MAX_FFT_F32 : CBP_MAX_FFT_F64; }

// ---------------------------------------------------------------- tuning
// Launch-shape knobs of one batch class, chosen by the autotuner.
struct tuning {
  int fold_rows;   // target rows per column-fold group (rounded up to a multiple of S; >= 32); 0: from the frame
  int cw;          // columns per column-pass strip (0: widest that fits and keeps >= 256 strips, one per CU)
  int wg_per_cu;   // persistent-grid cap of the streaming queues, workgroups per CU (0: one per item)
  int fft_order;   // radix pass order of the row and column FFTs
};
constexpr tuning kDefaultTuning = {0, 0, 0, 0};
// Row-pass items (one per (channel, fold group, residue)) a frame aims at
// when fold_rows is 0: one frame alone still spreads over the chip, a large
// frame keeps the fold's partial sums (one row per item) small.  The group
// depends on the frame alone, so a frame gets the same bits in any batch.
constexpr int kRowItemsPerFrame = 384;
constexpr int kRowWgPerCu = 4;   // resident inverse-row workgroups per CU (LDS: a row and its pass twiddle tables)

// Does a strip of cw columns of length Py fit the column pass?
bool col_fits(int Py, int cw, int twn, int esize) {
  return col_lds_bytes(Py, cw, twn, esize) <= kLdsLimit - 4096 && (int64_t)cw * Py <= col_max_strip_elems(esize);
}

// Columns per column-pass strip: `want` (a power of two up to 16) if given,
// else the widest strip of a workgroup of at most 512 threads (two or more per CU) that still
// leaves at least 256 strips over the frame's channels; either way narrowed
// until the strip fits.
int choose_cw(int Py, int hx, int nch, int twn, int esize, int want) {
  int cw = want > 0 ? want : 8;
  if (cw > 16) cw = 16;
  while (cw & (cw - 1)) cw &= cw - 1;
  while (cw > 1 && (!col_fits(Py, cw, twn, esize) ||
                    (want <= 0 && (col_threads(Py, cw, esize) > 512 ||
                                   (int64_t)((hx + cw - 1) / cw) * nch < 256))))
    cw >>= 1;
  return cw;
}

bool valid_image(const cbp_image* im) {
  if (!im || !im->data) return false;
  if (im->dtype != CBP_F32 && im->dtype != CBP_F64) return false;
  if (im->height < 1 || im->width < 1 || im->channels < 1) return false;
  if (im->pitch < im->width) return false;
  if (im->channels > 1 && im->channel_stride < (int64_t)im->height * im->pitch) return false;
  return true;
}

// An 8-bit stream (the quantisation entry points only).
bool valid_u8_image(const cbp_image* im) {
  if (!im || !im->data || im->dtype != CBP_U8) return false;
  if (im->height < 1 || im->width < 1 || im->channels < 1 || im->pitch < im->width) return false;
  if (im->channels > 1 && im->channel_stride < (int64_t)im->height * im->pitch) return false;
  return true;
}

cbp_status check_options(const cbp_options* o, int dtype) {
  if (!o) return CBP_E_INVALID;
  if ((o->learned != 0) != (o->mlp_blob != nullptr)) return CBP_E_INVALID;   // the learned form needs its network
  if (!(o->lambda >= 0.0) || o->tau != 0.0 || (o->flags & ~kKnownFlags) != 0) return CBP_E_INVALID;
  // one scale fix at a time; the learned form has its own weighted one
  if ((o->flags & CBP_FLAG_SCALE_K1) && (o->flags & CBP_FLAG_ONE_AXIS)) return CBP_E_INVALID;
  if (o->learned && (o->flags & (CBP_FLAG_SCALE_K1 | CBP_FLAG_ONE_AXIS))) return CBP_E_UNSUPPORTED;
  if (o->precision == CBP_PREC_FP64) return dtype == CBP_F64 ? CBP_OK : CBP_E_INVALID;
  if (o->precision == CBP_PREC_MIXED || o->precision == CBP_PREC_MFMA32 || o->precision == CBP_PREC_BF16 ||
      o->precision == CBP_PREC_MFMA64)
    return dtype == CBP_F32 ? CBP_OK : CBP_E_INVALID;
  return CBP_E_INVALID;
}

// Gram route of a precision form: -1 = double-double correlations (FP64,
// MIXED), 0 = matrix cores on FP32 operands (MFMA32), 1 = on bfloat16 (BF16),
// 2 = FP64 matrix cores on the FP64 evaluations (MFMA64).
int gram_format(int precision) {
  return precision == CBP_PREC_MFMA32 ? 0 : precision == CBP_PREC_BF16 ? 1 : precision == CBP_PREC_MFMA64 ? 2 : -1;
}

// Shapes -> plan.  All checks are host-side.
// sizes_only: the plan of the size-estimation entry point, which runs only
// the evaluation and the Gram (any S >= 1; no FFT or solver limits).
cbp_status make_plan(const cbp_image* b1, const cbp_image* b2, int m, int n, const cbp_options* o,
                     const tuning& tn, frame_plan* fp, bool sizes_only = false) {
  if (!valid_image(b1) || !valid_image(b2)) return CBP_E_INVALID;
  if (b1->dtype != b2->dtype || b1->channels != b2->channels) return CBP_E_INVALID;
  const cbp_status so = check_options(o, b1->dtype);
  if (so != CBP_OK) return so;
  if (m < 1 || n < 1) return CBP_E_SHAPE;
  const int k1 = b1->height - m + 1, k2 = b2->height - m + 1;
  if (b1->width - n + 1 != k1 || b2->width - n + 1 != k2) return CBP_E_SHAPE;
  if (k1 < 1 || k2 < 1 || k1 > CBP_MAX_K || k2 > CBP_MAX_K) return CBP_E_SHAPE;
  const int kmax = k1 > k2 ? k1 : k2;
  const int S = o->samples ? o->samples : kmax;
  if (S < (sizes_only ? 1 : kmax) || S > CBP_MAX_S) return CBP_E_INVALID;
  // the one-axis scale fix needs at least S - 1 support equations
  if (!sizes_only && (o->flags & CBP_FLAG_ONE_AXIS) && k1 * (S - k1) + k2 * (S - k2) < S - 1) return CBP_E_INVALID;
  const int esize = b1->dtype == CBP_F32 ? 4 : 8;
  fp->H1 = b1->height; fp->W1 = b1->width; fp->H2 = b2->height; fp->W2 = b2->width;
  fp->Hmax = fp->H1 > fp->H2 ? fp->H1 : fp->H2;
  fp->Wmax = fp->W1 > fp->W2 ? fp->W1 : fp->W2;
  fp->m = m; fp->n = n; fp->k1 = k1; fp->k2 = k2; fp->S = S; fp->N = k1 + k2;
  fp->nch = b1->channels;
  // rows of one residue per fold group (each a row-pass item): at least
  // 32 / S (the workspace's bound on the groups)
  int gi = (32 + S - 1) / S;
  if (tn.fold_rows > 0) gi = std::max(gi, (tn.fold_rows + S - 1) / S);
  else gi = std::max(gi, fp->nch * fp->Hmax / kRowItemsPerFrame);
  fp->rpg = S * gi;
  fp->RG = (fp->Hmax + fp->rpg - 1) / fp->rpg;
  fp->Py = smooth7(fp->Hmax);
  fp->Px = smooth7(fp->Wmax);
  if (sizes_only) {
    fp->hx = fp->Px / 2 + 1;
    fp->hxp = pitch_of(fp->hx, esize);
    fp->cw = 1;
    layout(fp, regions(fp->Hmax, fp->Wmax, kmax, S, fp->nch, esize));
    return CBP_OK;
  }
  if (fp->Py > max_fft(esize) || fp->Px > max_fft(esize)) return CBP_E_SHAPE;
  if (!make_fft_plan(fp->Py, &fp->fy, tn.fft_order) || !make_fft_plan(fp->Px, &fp->fx, tn.fft_order, true))
    return CBP_E_SHAPE;
  fp->hx = fp->Px / 2 + 1;
  fp->hxp = pitch_of(fp->hx, esize);
  fp->twy = col_table_entries(fp->fy);
  fp->twx = pass_table_entries(fp->fx);
  fp->cw = choose_cw(fp->Py, fp->hx, fp->nch, fp->twy, esize, tn.cw);
  const int gfmt = gram_format(o->precision);
  if (gfmt >= 0 && (fp->N > 32 || gram_mfma_lds_bytes(std::max(fp->Hmax, fp->Wmax), gfmt) > kLdsLimit - 2048))
    return CBP_E_UNSUPPORTED;
  if (o->learned && fp->N > 32) return CBP_E_UNSUPPORTED;   // 32 spectrum features per sample
  if (sample_lds_bytes(fp->N) > kLdsLimit - 2048 || finalize_lds_bytes(S, o->learned != 0) > kLdsLimit - 2048 ||
      row_lds_bytes(fp->Px, fp->twx, esize) > kLdsLimit - 2048 || !col_fits(fp->Py, fp->cw, fp->twy, esize))
    return CBP_E_SHAPE;
  layout(fp, regions(fp->Hmax, fp->Wmax, kmax, S, fp->nch, esize));
  return CBP_OK;
}

frame_desc make_desc(const frame_plan& fp, const cbp_image* b1, const cbp_image* b2, char* ws, double* K1,
                     double* K2, const cbp_image* latent, double lambda, void* diag, bool learned, int variant) {
  frame_desc d;
  std::memset(&d, 0, sizeof d);
  d.b1 = b1->data;
  d.b2 = b2->data;
  d.p1 = b1->pitch;
  d.p2 = b2->pitch;
  d.cs1 = b1->channels > 1 ? b1->channel_stride : 0;
  d.cs2 = b2->channels > 1 ? b2->channel_stride : 0;
  d.H1 = fp.H1; d.W1 = fp.W1; d.H2 = fp.H2; d.W2 = fp.W2; d.Hmax = fp.Hmax; d.Wmax = fp.Wmax;
  d.nch = fp.nch;
  d.ncf = 2 * fp.nch;
  d.m = fp.m; d.n = fp.n; d.k1 = fp.k1; d.k2 = fp.k2; d.S = fp.S; d.N = fp.N;
  d.rpg = fp.rpg; d.RG = fp.RG; d.Py = fp.Py; d.Px = fp.Px; d.hx = fp.hx; d.cw = fp.cw;
  d.hxp = fp.hxp;
  d.fy = fp.fy;
  d.fx = fp.fx;
  d.fpart = (double*)(ws + fp.off_fpart);
  d.ex = (c64*)(ws + fp.off_ex);
  d.ey = (c64*)(ws + fp.off_ey);
  d.corr = (cdd*)(ws + fp.off_corr);
  d.xvec = (c64*)(ws + fp.off_xvec);
  d.pq = (c64*)(ws + fp.off_pq);
  d.t1 = ws + fp.off_t1;
  d.t2 = ws + fp.off_t2;
  d.u = ws + fp.off_u;
  d.K1 = K1 ? K1 : (double*)(ws + fp.off_kern);
  d.K2 = K2 ? K2 : (double*)(ws + fp.off_kern) + CBP_MAX_K * CBP_MAX_K;
  if (latent) {
    d.out = latent->data;
    d.opitch = latent->pitch;
    d.ocs = latent->channels > 1 ? latent->channel_stride : 0;
  }
  d.lambda = lambda;
  d.diag = (cbp_diag*)diag;
  d.feat = (learned || diag) ? (float*)(ws + fp.off_feat) : nullptr;
  d.wts = learned ? (double*)(ws + fp.off_wts) : nullptr;
  d.Kalt = (double*)(ws + fp.off_kalt);
  d.twxd = (c64*)(ws + fp.off_twxd);
  d.kr = ws + fp.off_kr;
  d.variant = variant;
  return d;
}

// ---------------------------------------------------------------- phase timing state
struct pending_pair {
  int phase;
  hipEvent_t a, b;
};

struct profiler {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<pending_pair> pending;
  hipEvent_t open[PH_COUNT] = {};
  double total[PH_COUNT] = {};
  int64_t count[PH_COUNT] = {};

  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

profiler& prof() {
  static profiler p;
  return p;
}

thread_local bool t_capturing = false;  // no timing events inside a graph capture

// The HIP call that made the last CBP_E_DEVICE of this thread (cbp_last_error).
thread_local char t_error[256] = "";

hipError_t note(const char* what, hipError_t e) {
  if (e != hipSuccess) std::snprintf(t_error, sizeof t_error, "%s: %s", what, hipGetErrorString(e));
  return e;
}
#define CBP_TRY(expr)                                     \
  do {                                                    \
    const hipError_t e_ = note(#expr, (expr));            \
    if (e_ != hipSuccess) return e_;                      \
  } while (0)

const char* kPhaseNames[PH_COUNT] = {"fold_cols", "eval_cols", "eval_rows", "gram", "sample_eig",
                                     "scale_assemble", "row_fft_fwd", "col_fft_filter", "row_fft_inv",
                                     "kernel_row_dft"};

// ---------------------------------------------------------------- per-device state
// Pinned host staging for the descriptor upload of an eager batched call;
// a slot is reused only after the copy recorded on it has completed.
struct pinned_slot {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool recorded = false;
};
constexpr int kRing = 16;

struct graph_entry {
  hipGraphExec_t exec = nullptr;
  void* host = nullptr;  // pinned copy of the workspace head the graph uploads on every replay
  uint64_t last_use = 0;
};
constexpr size_t kMaxGraphs = 64;

// Capture stream, events, staging ring, graph and tuning caches of one
// device (created once; every stream at the default priority).  A call's
// kernels all run in order on the caller's stream: running the row pass on a
// second stream beside the column fold -> Gram chain measured slower than the
// plain order, the two cross-stream event waits costing more than the
// overlap gained.
struct dev_state {
  std::mutex launch_mu;  // one launch sequence at a time per device (the events are shared)
  bool ready = false;
  hipStream_t cap = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  pinned_slot ring[kRing];
  int next = 0;
  std::map<std::string, graph_entry> graphs;
  uint64_t tick = 0;
  std::map<std::string, tuning> tuned;
  bool have_last = false;
  cbp_tuning last = {};
  void* scratch = nullptr;   // this device's copy of `scratch` (device address)
};

dev_state* get_dev() {
  static std::mutex mu;
  static dev_state states[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  dev_state& f = states[dev];
  if (!f.ready) {
    if (note("hipStreamCreateWithFlags", hipStreamCreateWithFlags(&f.cap, hipStreamNonBlocking)) != hipSuccess ||
        note("hipEventCreate", hipEventCreate(&f.t0)) != hipSuccess ||
        note("hipEventCreate", hipEventCreate(&f.t1)) != hipSuccess)
      return nullptr;
    for (pinned_slot& s : f.ring)
      if (note("hipEventCreateWithFlags", hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess)
        return nullptr;
    if (note("hipGetSymbolAddress", hipGetSymbolAddress(&f.scratch, HIP_SYMBOL(scratch))) != hipSuccess ||
        f.scratch == nullptr)
      return nullptr;
    set_recover_attrs();
    set_fft_attrs();
    set_gram_mfma_attrs();
    set_size_attrs();
    set_encoder_attrs();
    f.ready = true;
  }
  return &f;
}

// ---------------------------------------------------------------- launch chain
// One launch of every queue over a set of frames: either one frame (one !=
// nullptr, descs == nullptr) or a chunk of a batch.
struct chunk_view {
  const frame_desc* descs;  // device
  const int* starts;        // device
  int* ctr;                 // device: the chunk's item counters
  int nf;
  int items[Q_COUNT];
  int grid[Q_COUNT];
  int maxN, maxS, maxPx, maxPy, maxcw;
  int maxTwx, maxTwy;   // largest row / column pass twiddle tables (entries)
  int colGroups;        // the column filter's row groups of the frames (bit g set for group g)
  int gram_fmt;   // gram_format() of the call's precision
  int maxStride;  // largest Hmax / Wmax (matrix-core Gram staging)
  bool finLean;   // no frame's scale solve refines or records diagnostics
  const void* mlp;  // the learned form's network (device mlp blob) or NULL
};

int grid_for(int items, int cap) {
  int g = items;
  if (cap > 0 && g > cap) g = cap;
  if (g >= 64) g = (g + 7) & ~7;  // a multiple of 8: XCD-aware item ranges
  return g < 1 ? 1 : g;
}

template <typename T>
hipError_t enqueue_chunk(dev_state& ds, const chunk_view& cv, bool latent, bool diag, hipStream_t st,
                         const inline_head* ih) {
  const batch_ref b = {cv.descs, cv.starts, cv.nf, cv.ctr};
  auto br = [&](int) { return b; };
  // the first launch (with an inline head it also stores the call's head):
  // a deblurring call's twiddle table of the kernels' row DFTs only, since
  // its row pass folds the columns; a kernel-only call's column fold
  CBP_TRY(launch_fold<T>(br(Q_FOLD), latent ? 0 : cv.grid[Q_FOLD], latent ? cv.grid[Q_TWID] : 0, ih, st));
  if (diag) CBP_TRY(launch_diag_init(br(Q_DIAG), cv.grid[Q_DIAG], st));
  // the row pass (with the column fold and the row evaluation) or the row
  // evaluation alone, then the column evaluation of the fold
  if (latent) CBP_TRY(launch_row_fwd<T>(br(Q_ROW_FWD), cv.grid[Q_ROW_FWD], cv.maxPx, cv.maxTwx, 1, st));
  else CBP_TRY(launch_eval_rows<T>(br(Q_EVAL_ROWS), cv.grid[Q_EVAL_ROWS], st));
  CBP_TRY(launch_eval_cols(br(Q_EVAL_COLS), cv.grid[Q_EVAL_COLS], st));
  // join: the Gram needs the row evaluation (and the column pass the row spectra)
  if (cv.gram_fmt < 0) CBP_TRY(launch_gram(br(Q_GRAM), cv.grid[Q_GRAM], st));
  else CBP_TRY(launch_gram_mfma(br(Q_GRAMM), cv.grid[Q_GRAMM], cv.gram_fmt, cv.maxStride, st));
  CBP_TRY(launch_sample(br(Q_SAMPLE), cv.grid[Q_SAMPLE], cv.maxN, st));
  if (cv.mlp) {
    // the learned form: plain kernels (the fallback), the network's weights,
    // the learned kernels, and the judge between them
    CBP_TRY(launch_finalize(br(Q_FINALIZE), cv.grid[Q_FINALIZE], cv.maxS, 0, 1, cv.finLean, st));
    CBP_TRY(launch_mlp_frames(br(Q_FINALIZE), cv.grid[Q_FINALIZE], cv.mlp, st));
    CBP_TRY(launch_finalize(br(Q_FINALIZE), cv.grid[Q_FINALIZE], cv.maxS, 1, 0, cv.finLean, st));
    CBP_TRY(launch_judge(br(Q_FINALIZE), cv.grid[Q_FINALIZE], st));
  } else {
    CBP_TRY(launch_finalize(br(Q_FINALIZE), cv.grid[Q_FINALIZE], cv.maxS, 0, 0, cv.finLean, st));
  }
  if (latent) {
    CBP_TRY(launch_kernel_dft<T>(br(Q_KRDFT), cv.grid[Q_KRDFT], st));
    CBP_TRY(launch_col<T>(br(Q_COL), cv.grid[Q_COL], cv.maxPy, cv.maxcw, cv.maxTwy, cv.colGroups, st));
    CBP_TRY(launch_row_inv<T>(br(Q_ROW_INV), cv.grid[Q_ROW_INV], cv.maxPx, cv.maxTwx, st));
  }
  return hipSuccess;
}

hipError_t enqueue(dev_state& ds, int dtype, const chunk_view& cv, bool latent, bool diag, hipStream_t st,
                   const inline_head* ih) {
  return dtype == CBP_F32 ? enqueue_chunk<float>(ds, cv, latent, diag, st, ih)
                          : enqueue_chunk<double>(ds, cv, latent, diag, st, ih);
}

// ---------------------------------------------------------------- batches
struct frame_req {
  const cbp_image* b1;
  const cbp_image* b2;
  cbp_image* latent;
  int m, n;
  double* K1;
  double* K2;
  void* diag;
};

// Plans, descriptors and launch shapes of the valid frames of one batch.
struct batch_build {
  int dtype = CBP_F32;
  bool latent = false, diag = false;
  std::vector<int> idx;            // request index of each valid frame
  std::vector<frame_plan> plans;
  std::vector<char> head;          // bytes uploaded to the workspace head
  std::vector<chunk_view> chunks;  // device pointers into the head
  char* head_dev = nullptr;
};

// Class of a batch for the tuning cache: dtype, frame count, latent, and the
// largest frame, kernel and channel count.
std::string class_key(const std::vector<frame_req>& reqs, const cbp_options* o) {
  int H = 0, W = 0, k = 0, ch = 0, dt = reqs.empty() ? 0 : reqs[0].b1->dtype;
  for (const frame_req& r : reqs) {
    H = std::max({H, r.b1->height, r.b2->height});
    W = std::max({W, r.b1->width, r.b2->width});
    k = std::max({k, r.b1->height - r.m + 1, r.b2->height - r.m + 1});
    ch = std::max(ch, r.b1->channels);
  }
  char buf[160];
  std::snprintf(buf, sizeof buf, "%d/%zu/%d/%d/%d/%d/%d/%d/%d", dt, reqs.size(), reqs.empty() ? 0 : reqs[0].latent != nullptr,
                H, W, k, ch, o->samples, o->precision);
  return buf;
}

// Validate and plan every frame; statuses go to `status` (one per request).
// Returns CBP_E_NOMEM when the valid frames do not fit the workspace.
cbp_status build_batch(const std::vector<frame_req>& reqs, const cbp_options* o, const tuning& tn,
                       std::vector<cbp_status>& status, batch_build* bb, bool sizes_only = false) {
  const int nreq = (int)reqs.size();
  status.assign(nreq, CBP_OK);
  bb->idx.clear();
  bb->plans.clear();
  bb->chunks.clear();
  const int dtype = reqs[0].b1 ? reqs[0].b1->dtype : -1;
  const bool latent = reqs[0].latent != nullptr;
  for (int f = 0; f < nreq; ++f) {
    const frame_req& r = reqs[f];
    frame_plan fp;
    cbp_status s = make_plan(r.b1, r.b2, r.m, r.n, o, tn, &fp, sizes_only);
    if (s == CBP_OK && r.b1->dtype != dtype) s = CBP_E_INVALID;
    if (s == CBP_OK && (r.latent != nullptr) != latent) s = CBP_E_INVALID;
    if (s == CBP_OK && latent &&
        (!valid_image(r.latent) || r.latent->dtype != dtype || r.latent->channels != r.b1->channels ||
         r.latent->height != r.m || r.latent->width != r.n))
      s = CBP_E_INVALID;
    status[f] = s;
    if (s == CBP_OK) {
      bb->idx.push_back(f);
      bb->plans.push_back(fp);
    }
  }
  const int nf = (int)bb->idx.size();
  bb->dtype = dtype;
  bb->latent = latent;
  bb->diag = o->diag != nullptr;
  if (nf == 0) return CBP_OK;
  const size_t head = head_bytes(nf);
  size_t need = head;
  for (const frame_plan& fp : bb->plans) need += fp.total;
  if (!o->workspace || o->workspace_bytes < need) {
    for (int f : bb->idx) status[f] = CBP_E_NOMEM;
    return CBP_E_NOMEM;
  }
  char* ws = (char*)o->workspace;
  bb->head_dev = ws;
  bb->head.assign(head, 0);
  frame_desc* descs = (frame_desc*)bb->head.data();
  int* starts = (int*)(bb->head.data() + head_desc_bytes(nf));
  size_t off = head;
  for (int i = 0; i < nf; ++i) {
    const frame_req& r = reqs[bb->idx[i]];
    descs[i] = make_desc(bb->plans[i], r.b1, r.b2, ws + off, r.K1, r.K2, r.latent, o->lambda, r.diag,
                         o->learned != 0,
                         variant_bits(o->flags) | (gram_format(o->precision) >= 0 ? VAR_FP64_GRAM : 0));
    off += bb->plans[i].total;
  }
  const int cap = tn.wg_per_cu > 0 ? tn.wg_per_cu * kComputeUnits : 0;
  for (int c = 0; c < nchunks(nf); ++c) {
    const int f0 = c * BATCH_CHUNK, cnt = std::min(BATCH_CHUNK, nf - f0);
    int* st = starts + (size_t)c * Q_COUNT * (BATCH_CHUNK + 1);
    chunk_view cv = {};
    cv.descs = (const frame_desc*)bb->head_dev + f0;
    cv.starts = (const int*)(bb->head_dev + head_desc_bytes(nf)) + (size_t)c * Q_COUNT * (BATCH_CHUNK + 1);
    cv.ctr = (int*)(bb->head_dev + head_desc_bytes(nf) + head_starts_bytes(nf)) + (size_t)c * CTR_COUNT;
    cv.nf = cnt;
    for (int q = 0; q < Q_COUNT; ++q) {
      // layout of one chunk's prefix sums: [Q][cnt + 1]
      int* sq = st + (size_t)q * (cnt + 1);
      sq[0] = 0;
      for (int i = 0; i < cnt; ++i) sq[i + 1] = sq[i] + queue_items(q, bb->plans[f0 + i]);
      cv.items[q] = sq[cnt];
      const bool streaming = q != Q_SAMPLE && q != Q_FINALIZE && q != Q_DIAG && q != Q_GRAMM;
      // the row passes always run a persistent grid (their workgroups load
      // the next rows while transforming the current ones)
      const bool row = q == Q_ROW_FWD || q == Q_ROW_INV;
      cv.grid[q] = grid_for(cv.items[q], row ? (cap > 0 ? cap : kRowWgPerCu * kComputeUnits) : streaming ? cap : 0);
    }
    cv.maxN = cv.maxS = cv.maxPx = cv.maxPy = cv.maxcw = cv.maxStride = 1;
    cv.colGroups = 0;
    cv.gram_fmt = gram_format(o->precision);
    cv.mlp = o->learned ? o->mlp_blob : nullptr;
    cv.finLean = true;
    for (int i = 0; i < cnt; ++i) {
      const frame_desc& fd = descs[f0 + i];
      cv.finLean = cv.finLean && solve_refine_max(fd.variant) == 0 && fd.diag == nullptr && !(fd.variant & VAR_ONE_AXIS);
      const frame_plan& p = bb->plans[f0 + i];
      cv.maxStride = std::max({cv.maxStride, p.Hmax, p.Wmax});
      cv.maxN = std::max(cv.maxN, p.N);
      cv.maxS = std::max(cv.maxS, p.S);
      cv.maxPx = std::max(cv.maxPx, p.Px);
      cv.maxPy = std::max(cv.maxPy, p.Py);
      cv.maxcw = std::max(cv.maxcw, p.cw);
      cv.maxTwx = std::max(cv.maxTwx, p.twx);
      cv.maxTwy = std::max(cv.maxTwy, p.twy);
      cv.colGroups |= 1 << col_group_size(p.Py);
    }
    const int esize = dtype == CBP_F32 ? 4 : 8;
    // as many persistent row-pass workgroups as stay resident
    if (cap == 0) cv.grid[Q_ROW_FWD] = grid_for(cv.items[Q_ROW_FWD], row_fwd_per_cu(row_lds_bytes(cv.maxPx, cv.maxTwx, esize), esize) * kComputeUnits);
    // the widest strip and the tallest column share one allocation; keep it in LDS
    while (cv.maxcw > 1 && !col_fits(cv.maxPy, cv.maxcw, cv.maxTwy, esize)) {
      cv.maxcw >>= 1;
      for (int i = 0; i < cnt; ++i) {
        frame_plan& p = bb->plans[f0 + i];
        if (p.cw > cv.maxcw) {
          p.cw = cv.maxcw;
          descs[f0 + i].cw = p.cw;
        }
      }
      int* sq = st + (size_t)Q_COL * (cnt + 1);
      for (int i = 0; i < cnt; ++i) sq[i + 1] = sq[i] + queue_items(Q_COL, bb->plans[f0 + i]);
      cv.items[Q_COL] = sq[cnt];
    }
    // the column pass runs a persistent grid: its workgroups load the next
    // strip while finishing the current one (as many as stay resident)
    cv.grid[Q_COL] = grid_for(cv.items[Q_COL],
                              cap > 0 ? cap : col_per_cu(cv.maxPy, cv.maxcw, cv.maxTwy, col_group_size(cv.maxPy), esize) * kComputeUnits);
    bb->chunks.push_back(cv);
  }
  return CBP_OK;
}

// Copy the workspace head from a pinned staging slot (asynchronous on st).
hipError_t upload_bytes(dev_state& ds, void* dst, const std::vector<char>& bytes, hipStream_t st) {
  pinned_slot& s = ds.ring[ds.next];
  ds.next = (ds.next + 1) % kRing;
  if (s.recorded) CBP_TRY(hipEventSynchronize(s.done));
  if (s.cap < bytes.size()) {
    if (s.host) (void)hipHostFree(s.host);
    s.host = nullptr;
    s.cap = 0;
    CBP_TRY(hipHostMalloc(&s.host, bytes.size(), hipHostMallocDefault));
    s.cap = bytes.size();
  }
  std::memcpy(s.host, bytes.data(), bytes.size());
  CBP_TRY(hipMemcpyAsync(dst, s.host, bytes.size(), hipMemcpyHostToDevice, st));
  CBP_TRY(hipEventRecord(s.done, st));
  s.recorded = true;
  return hipSuccess;
}

hipError_t upload_head(dev_state& ds, const batch_build& bb, hipStream_t st) {
  return upload_bytes(ds, bb.head_dev, bb.head, st);
}

hipError_t enqueue_batch(dev_state& ds, const batch_build& bb, hipStream_t st, const inline_head* ih = nullptr) {
  for (const chunk_view& cv : bb.chunks) {
    const hipError_t e = enqueue(ds, bb.dtype, cv, bb.latent, bb.diag, st, ih);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The head of a one-chunk call of at most three frames as an inline head (the
// descriptors, then the chunk's prefix sums); false when it does not fit.
bool make_inline_head(const batch_build& bb, inline_head* ih) {
  if (bb.chunks.size() != 1) return false;
  const int nf = bb.chunks[0].nf;
  // the prefix sums travel in whole 16-byte units (the kernel copies them so);
  // the padding lands in the workspace head's prefix-sum region, which is larger
  const size_t nd = (size_t)nf * sizeof(frame_desc), ns = (size_t)Q_COUNT * (nf + 1) * sizeof(int);
  const size_t nsp = (ns + 15) & ~(size_t)15;
  if (nd % 16 != 0 || nd + nsp > (size_t)kInlineHeadMax) return false;
  ih->ndesc_bytes = (int)nd;
  ih->nstart_bytes = (int)nsp;
  std::memcpy(ih->bytes, bb.head.data(), nd);
  std::memcpy(ih->bytes + nd, bb.head.data() + head_desc_bytes(nf), ns);
  std::memset(ih->bytes + nd + ns, 0, nsp - ns);
  return true;
}

// Key of a captured graph: everything its nodes bake in.
std::string graph_key(const batch_build& bb) {
  std::string k(bb.head.begin(), bb.head.end());
  for (const chunk_view& cv : bb.chunks) k.append((const char*)&cv, sizeof cv);
  k.append((const char*)&bb.head_dev, sizeof bb.head_dev);
  k.push_back((char)bb.dtype);
  k.push_back((char)bb.latent);
  k.push_back((char)bb.diag);
  return k;   // the chunk views carry the network pointer
}

hipError_t run_graph(dev_state& ds, const batch_build& bb, hipStream_t st) {
  const std::string key = graph_key(bb);
  auto it = ds.graphs.find(key);
  hipError_t e;
  if (it == ds.graphs.end()) {
    if (ds.graphs.size() >= kMaxGraphs) {
      // evict the least recently used graph once the caller's work has drained
      auto lru = ds.graphs.begin();
      for (auto g = ds.graphs.begin(); g != ds.graphs.end(); ++g)
        if (g->second.last_use < lru->second.last_use) lru = g;
      if ((e = note("hipDeviceSynchronize", hipDeviceSynchronize())) != hipSuccess) return e;
      hipGraphExecDestroy(lru->second.exec);
      hipHostFree(lru->second.host);
      ds.graphs.erase(lru);
    }
    graph_entry ent;
    if ((e = note("hipHostMalloc", hipHostMalloc(&ent.host, bb.head.size(), hipHostMallocDefault))) != hipSuccess)
      return e;
    std::memcpy(ent.host, bb.head.data(), bb.head.size());
    hipGraph_t g = nullptr;
    if ((e = note("hipStreamBeginCapture", hipStreamBeginCapture(ds.cap, hipStreamCaptureModeRelaxed))) !=
        hipSuccess) {
      hipHostFree(ent.host);
      return e;
    }
    t_capturing = true;
    // a small head rides in the first launch's arguments (baked into the
    // graph; the key covers the head's bytes), else a copy node uploads it
    inline_head ih;
    hipError_t ce;
    if (make_inline_head(bb, &ih)) {
      ce = enqueue_batch(ds, bb, ds.cap, &ih);
    } else {
      ce = note("hipMemcpyAsync (capture)",
                hipMemcpyAsync(bb.head_dev, ent.host, bb.head.size(), hipMemcpyHostToDevice, ds.cap));
      if (ce == hipSuccess) ce = enqueue_batch(ds, bb, ds.cap);
    }
    t_capturing = false;
    e = note("hipStreamEndCapture", hipStreamEndCapture(ds.cap, &g));
    if (ce == hipSuccess && e == hipSuccess)
      e = note("hipGraphInstantiate", hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0));
    if (g) hipGraphDestroy(g);
    if (ce != hipSuccess || e != hipSuccess) {
      hipHostFree(ent.host);
      return ce != hipSuccess ? ce : e;
    }
    it = ds.graphs.emplace(key, ent).first;
  }
  it->second.last_use = ++ds.tick;
  return note("hipGraphLaunch", hipGraphLaunch(it->second.exec, st));
}

// Time one eager run of a batch with tuning tn (ms; < 0 on failure).
float time_tuning(dev_state& ds, const std::vector<frame_req>& reqs, const cbp_options* o, const tuning& tn,
                  hipStream_t st) {
  std::vector<cbp_status> status;
  batch_build bb;
  if (build_batch(reqs, o, tn, status, &bb) != CBP_OK || bb.idx.empty()) return -1.0f;
  if (upload_head(ds, bb, st) != hipSuccess) return -1.0f;
  if (enqueue_batch(ds, bb, st) != hipSuccess) return -1.0f;  // warm-up
  float best = -1.0f;
  for (int rep = 0; rep < 5; ++rep) {
    if (hipEventRecord(ds.t0, st) != hipSuccess) return -1.0f;
    if (enqueue_batch(ds, bb, st) != hipSuccess) return -1.0f;
    if (hipEventRecord(ds.t1, st) != hipSuccess) return -1.0f;
    float ms = 0.0f;
    if (hipEventSynchronize(ds.t1) != hipSuccess || hipEventElapsedTime(&ms, ds.t0, ds.t1) != hipSuccess)
      return -1.0f;
    if (best < 0.0f || ms < best) best = ms;
  }
  return best;
}

// Coordinate search over the knobs, one at a time, from the defaults.  A
// candidate replaces the best shape only when it is faster by more than
// kTuneMargin, so that timing noise does not pick between equals.
constexpr float kTuneMargin = 0.01f;
tuning autotune(dev_state& ds, const std::vector<frame_req>& reqs, const cbp_options* o, hipStream_t st,
                float* best_ms) {
  tuning best = kDefaultTuning;
  float bms = time_tuning(ds, reqs, o, best, st);
  auto consider = [&](tuning t) {
    const float ms = time_tuning(ds, reqs, o, t, st);
    if (ms > 0.0f && (bms < 0.0f || ms < bms * (1.0f - kTuneMargin))) {
      bms = ms;
      best = t;
    }
  };
  for (int order = 1; order < FFT_ORDERS; ++order) { tuning t = best; t.fft_order = order; consider(t); }
  for (int rows : {32, 64, 128, 256}) { tuning t = best; t.fold_rows = rows; consider(t); }
  for (int cw : {1, 2, 4, 8, 16}) { tuning t = best; t.cw = cw; consider(t); }
  for (int wpc : {2, 4, 8, 16}) { tuning t = best; t.wg_per_cu = wpc; consider(t); }
  *best_ms = bms;
  return best;
}

// Candidates of a size search (as the oracle forms them): k1' = kmin, kmin +
// step, ... <= kmax with 1 <= k1' - d, both trial sizes <= CBP_MAX_K and
// k1' <= min(H1, W1).  False for a malformed search.
bool size_candidates(int d, const cbp_size_search* s, int H1, int W1, size_cands* c) {
  if (s->kmin < 1 || s->kmax < s->kmin || s->step < 1) return false;
  c->n = 0;
  c->d = d;
  for (int k = s->kmin; k <= s->kmax && c->n < CBP_MAX_K; k += s->step)
    if (k - d >= 1 && k <= CBP_MAX_K && k - d <= CBP_MAX_K && k <= H1 && k <= W1) c->k1[c->n++] = k;
  return true;
}

size_t size_ratio_bytes(int ncand, int S) { return align_up((size_t)ncand * 2 * S * sizeof(double)); }

// no_alloc: the call must not allocate (the allocation-free entry point):
// its head has to travel inline, never through a pinned staging copy.
cbp_status batch_call(const std::vector<frame_req>& reqs, cbp_status* per_frame, const cbp_options* o,
                      bool no_alloc = false) {
  if (reqs.empty() || !o) return CBP_E_INVALID;
  for (const frame_req& r : reqs)
    if (!r.b1 || !r.b2) return CBP_E_INVALID;
  // host validation first (no HIP call when every frame is invalid)
  std::vector<cbp_status> status;
  batch_build bb;
  cbp_status s = build_batch(reqs, o, kDefaultTuning, status, &bb);
  if (per_frame)
    for (size_t f = 0; f < reqs.size(); ++f) per_frame[f] = status[f];
  cbp_status first = CBP_OK;
  for (cbp_status x : status)
    if (x != CBP_OK) { first = x; break; }
  if (s != CBP_OK || bb.idx.empty()) return s != CBP_OK ? s : first;
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  hipStream_t st = (hipStream_t)o->stream;
  std::lock_guard<std::mutex> lk(ds->launch_mu);
  (void)hipGetLastError();  // launch errors below are read with hipGetLastError: start clean
  const std::string ck = class_key(reqs, o);
  auto tt = ds->tuned.find(ck);
  tuning tn = kDefaultTuning;
  if (tt != ds->tuned.end()) {
    tn = tt->second;
  } else if ((o->flags & CBP_FLAG_AUTOTUNE) && bb.idx.size() == reqs.size()) {
    // the search runs only on batches that are valid as given
    float ms = -1.0f;
    tn = autotune(*ds, reqs, o, st, &ms);
    ds->tuned[ck] = tn;
    ds->have_last = true;
    ds->last = cbp_tuning{tn.fold_rows, tn.cw, tn.wg_per_cu, tn.fft_order, (double)ms};
  }
  if (std::memcmp(&tn, &kDefaultTuning, sizeof tn) != 0) {
    s = build_batch(reqs, o, tn, status, &bb);
    if (s != CBP_OK) return s;
  }
  hipError_t e;
  if (o->flags & CBP_FLAG_GRAPH) {
    e = run_graph(*ds, bb, st);
  } else {
    inline_head ih;
    if (make_inline_head(bb, &ih)) {
      e = enqueue_batch(*ds, bb, st, &ih);
    } else if (no_alloc) {
      return CBP_E_UNSUPPORTED;
    } else {
      e = upload_head(*ds, bb, st);
      if (e == hipSuccess) e = enqueue_batch(*ds, bb, st);
    }
  }
  if (e != hipSuccess) return CBP_E_DEVICE;
  return first;
}

}  // namespace

void prof_begin(int phase, hipStream_t st) {
  profiler& p = prof();
  if (!p.on || t_capturing) return;
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t e = p.get();
  if (!e) return;
  hipEventRecord(e, st);
  p.open[phase] = e;
}

void prof_end(int phase, hipStream_t st) {
  profiler& p = prof();
  if (!p.on || t_capturing) return;
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t a = p.open[phase];
  if (!a) return;
  hipEvent_t b = p.get();
  if (!b) return;
  hipEventRecord(b, st);
  p.pending.push_back({phase, a, b});
  p.open[phase] = nullptr;
}

}  // namespace cbp

using namespace cbp;

extern "C" {

const char* cbp_status_string(cbp_status s) {
  switch (s) {
    case CBP_OK: return "ok";
    case CBP_E_INVALID: return "invalid argument";
    case CBP_E_SHAPE: return "inconsistent or unsupported shape";
    case CBP_E_DEGENERATE: return "degenerate input";
    case CBP_E_DEVICE: return "device error";
    case CBP_E_NOMEM: return "workspace too small";
    case CBP_E_UNSUPPORTED: return "unsupported option";
  }
  return "unknown status";
}

const char* cbp_version(void) { return "0.2.0"; }

size_t cbp_diag_size(void) { return sizeof(cbp_diag); }

size_t cbp_workspace_size(int32_t maxH, int32_t maxW, int32_t maxk, int32_t channels, int32_t batch,
                          const cbp_options* opts) {
  if (maxH < 1 || maxW < 1 || maxk < 1 || maxk > CBP_MAX_K || channels < 1 || batch < 1) return 0;
  int S = maxk;
  int esize = 8;
  if (opts) {
    if (opts->samples > S) S = opts->samples;
    if (opts->precision != CBP_PREC_FP64) esize = 4;
  }
  if (S > CBP_MAX_S) return 0;
  frame_plan fp;
  const size_t one = layout(&fp, regions(maxH, maxW, maxk, S, channels, esize));
  return head_bytes(batch) + one * (size_t)batch;
}

cbp_status cbp_eval_unit_circle(const cbp_image* b, int32_t S, double* ex, double* ey, const cbp_options* opts) {
  if (!valid_image(b) || !ex || !ey || !opts) return CBP_E_INVALID;
  if (S < 1 || S > CBP_MAX_S) return CBP_E_INVALID;
  // one frame through the evaluation kernels: a one-slot (ncf = 1) descriptor
  // whose EX / EY are the caller's buffers; its fold partials follow the head
  frame_desc d;
  std::memset(&d, 0, sizeof d);
  d.b1 = d.b2 = b->data;
  d.p1 = d.p2 = b->pitch;
  d.H1 = d.H2 = d.Hmax = b->height;
  d.W1 = d.W2 = d.Wmax = b->width;
  d.nch = 1;
  d.ncf = 1;
  d.S = S;
  d.rpg = S * ((32 + S - 1) / S);
  d.RG = (b->height + d.rpg - 1) / d.rpg;
  const size_t head = head_bytes(1);
  const size_t need = head + ((size_t)(b->height + 31) / 32 + 1) * (size_t)S * b->width * sizeof(double);
  if (!opts->workspace || opts->workspace_bytes < need) return CBP_E_NOMEM;
  char* ws = (char*)opts->workspace;
  d.fpart = (double*)(ws + head);
  d.ex = (c64*)ex;
  d.ey = (c64*)ey;
  int items[Q_COUNT] = {};
  items[Q_FOLD] = ((d.Wmax + 63) / 64) * S * d.RG;
  items[Q_EVAL_COLS] = (d.Wmax + 15) / 16;
  items[Q_EVAL_ROWS] = (d.Hmax + 1) / 2;   // as queue_items, one (channel, frame) slot
  std::vector<char> hb(head, 0);
  std::memcpy(hb.data(), &d, sizeof d);
  int* starts = (int*)(hb.data() + head_desc_bytes(1));
  for (int q = 0; q < Q_COUNT; ++q) { starts[q * 2] = 0; starts[q * 2 + 1] = items[q]; }
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  hipStream_t st = (hipStream_t)opts->stream;
  const batch_ref br = {(const frame_desc*)ws, (const int*)(ws + head_desc_bytes(1)), 1, nullptr};
  std::lock_guard<std::mutex> lk(ds->launch_mu);
  (void)hipGetLastError();
  auto run = [&]() -> hipError_t {
    CBP_TRY(upload_bytes(*ds, ws, hb, st));
    if (b->dtype == CBP_F32) CBP_TRY(launch_fold<float>(br, grid_for(items[Q_FOLD], 0), 0, nullptr, st));
    else CBP_TRY(launch_fold<double>(br, grid_for(items[Q_FOLD], 0), 0, nullptr, st));
    CBP_TRY(launch_eval_cols(br, grid_for(items[Q_EVAL_COLS], 0), st));
    if (b->dtype == CBP_F32) CBP_TRY(launch_eval_rows<float>(br, grid_for(items[Q_EVAL_ROWS], 0), st));
    else CBP_TRY(launch_eval_rows<double>(br, grid_for(items[Q_EVAL_ROWS], 0), st));
    return hipSuccess;
  };
  return run() == hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_recover_kernels(const cbp_image* b1, const cbp_image* b2, int32_t m, int32_t n, double* K1,
                               double* K2, const cbp_options* opts) {
  if (!K1 || !K2 || !opts || !b1 || !b2) return CBP_E_INVALID;
  const std::vector<frame_req> reqs = {frame_req{b1, b2, nullptr, m, n, K1, K2, opts->diag}};
  return batch_call(reqs, nullptr, opts);
}

cbp_status cbp_deblur(const cbp_image* b1, const cbp_image* b2, cbp_image* latent, double* K1, double* K2,
                      const cbp_options* opts) {
  if (!opts || !latent || !b1 || !b2) return CBP_E_INVALID;
  const std::vector<frame_req> reqs = {frame_req{b1, b2, latent, latent->height, latent->width, K1, K2, opts->diag}};
  return batch_call(reqs, nullptr, opts);
}

cbp_status cbp_sample_grams(const cbp_image* b1, const cbp_image* b2, int32_t m, int32_t n, double* grams,
                            const cbp_options* opts) {
  if (!grams || !opts || !b1 || !b2) return CBP_E_INVALID;
  const std::vector<frame_req> reqs = {frame_req{b1, b2, nullptr, m, n, nullptr, nullptr, nullptr}};
  std::vector<cbp_status> status;
  batch_build bb;
  const cbp_status s = build_batch(reqs, opts, kDefaultTuning, status, &bb);
  if (s != CBP_OK) return s;
  if (status[0] != CBP_OK) return status[0];
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  const chunk_view& cv = bb.chunks[0];
  const batch_ref br = {cv.descs, cv.starts, cv.nf, cv.ctr};
  hipStream_t st = (hipStream_t)opts->stream;
  std::lock_guard<std::mutex> lk(ds->launch_mu);
  (void)hipGetLastError();
  auto run = [&]() -> hipError_t {
    CBP_TRY(upload_head(*ds, bb, st));
    if (b1->dtype == CBP_F32) {
      CBP_TRY(launch_fold<float>(br, cv.grid[Q_FOLD], 0, nullptr, st));
      CBP_TRY(launch_eval_rows<float>(br, cv.grid[Q_EVAL_ROWS], st));
    } else {
      CBP_TRY(launch_fold<double>(br, cv.grid[Q_FOLD], 0, nullptr, st));
      CBP_TRY(launch_eval_rows<double>(br, cv.grid[Q_EVAL_ROWS], st));
    }
    CBP_TRY(launch_eval_cols(br, cv.grid[Q_EVAL_COLS], st));
    if (cv.gram_fmt < 0) CBP_TRY(launch_gram(br, cv.grid[Q_GRAM], st));
    else CBP_TRY(launch_gram_mfma(br, cv.grid[Q_GRAMM], cv.gram_fmt, cv.maxStride, st));
    CBP_TRY(launch_gram_expand(br, cv.grid[Q_GRAMM], grams, st));
    return hipSuccess;
  };
  return run() == hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_deblur_batch(int32_t nframes, const cbp_image* b1s, const cbp_image* b2s, cbp_image* latents,
                            double* const* K1s, double* const* K2s, cbp_status* per_frame, const cbp_options* opts) {
  if (nframes < 1 || !b1s || !b2s || !latents || !opts) return CBP_E_INVALID;
  std::vector<frame_req> reqs(nframes);
  for (int f = 0; f < nframes; ++f)
    reqs[f] = frame_req{&b1s[f], &b2s[f], &latents[f], latents[f].height, latents[f].width,
                        K1s ? K1s[f] : nullptr, K2s ? K2s[f] : nullptr,
                        opts->diag ? (void*)((cbp_diag*)opts->diag + f) : nullptr};
  return batch_call(reqs, per_frame, opts);
}

cbp_status cbp_deblur_noalloc(const cbp_image* b1, const cbp_image* b2, cbp_image* latent, double* K1, double* K2,
                              const cbp_options* opts) {
  if (!opts || !latent || !b1 || !b2) return CBP_E_INVALID;
  // graphs pin a host copy of their head and the autotuner stages uploads:
  // both allocate, so neither is offered here
  if (opts->flags & (CBP_FLAG_GRAPH | CBP_FLAG_AUTOTUNE)) return CBP_E_UNSUPPORTED;
  // host validation and the scratch bound first (no HIP call before them)
  frame_plan fp;
  const cbp_status s = make_plan(b1, b2, latent->height, latent->width, opts, kDefaultTuning, &fp);
  if (s != CBP_OK) return s;
  const size_t need = head_bytes(1) + fp.total;
  if (need > kScratchBytes) {
    std::snprintf(t_error, sizeof t_error, "cbp_deblur_noalloc: the frame needs %zu bytes of scratch, the limit is %zu",
                  need, kScratchBytes);
    return CBP_E_NOMEM;
  }
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  // the one-frame head always travels in the first launch's arguments, so
  // the call makes no staging copy; the workspace is this device's scratch
  cbp_options o = *opts;
  o.workspace = ds->scratch;
  o.workspace_bytes = kScratchBytes;
  const std::vector<frame_req> reqs = {frame_req{b1, b2, latent, latent->height, latent->width, K1, K2, o.diag}};
  return batch_call(reqs, nullptr, &o, true);
}

size_t cbp_noalloc_scratch_bytes(void) { return kScratchBytes; }

size_t cbp_size_workspace_size(int32_t maxH, int32_t maxW, int32_t channels, int32_t d,
                               const cbp_size_search* search, const cbp_options* opts) {
  if (!search || maxH < 1 || maxW < 1 || channels < 1) return 0;
  size_cands c;
  if (!size_candidates(d, search, maxH, maxW, &c) || c.n == 0) return 0;
  const int K1 = c.k1[c.n - 1], kmax = std::max(K1, K1 - d);
  const int S = search->samples ? search->samples : K1;
  if (S < 1 || S > CBP_MAX_S) return 0;
  const int esize = (opts && opts->precision != CBP_PREC_FP64) ? 4 : 8;
  frame_plan fp;
  return head_bytes(1) + layout(&fp, regions(maxH, maxW, kmax, S, channels, esize)) + size_ratio_bytes(c.n, S);
}

cbp_status cbp_estimate_kernel_sizes(const cbp_image* b1, const cbp_image* b2, const cbp_size_search* search,
                                     cbp_size_result* result, double* ratios, const cbp_options* opts) {
  if (!b1 || !b2 || !search || !result || !opts) return CBP_E_INVALID;
  if (!valid_image(b1) || !valid_image(b2) || b1->dtype != b2->dtype || b1->channels != b2->channels)
    return CBP_E_INVALID;
  if (opts->precision != CBP_PREC_FP64 && opts->precision != CBP_PREC_MIXED) return CBP_E_INVALID;
  const int d = b1->height - b2->height;
  if (b1->width - b2->width != d) return CBP_E_SHAPE;
  size_cands c;
  if (!size_candidates(d, search, b1->height, b1->width, &c)) return CBP_E_INVALID;
  if (c.n == 0) return CBP_E_SHAPE;
  const int K1 = c.k1[c.n - 1];
  const int S = search->samples ? search->samples : K1;
  if (S < 1 || S > CBP_MAX_S) return CBP_E_INVALID;
  // the frame's plan at the largest trial sizes: its evaluation and Gram
  // correlations serve every candidate
  cbp_options o = *opts;
  o.samples = S;
  o.lambda = 0.0;
  o.tau = 0.0;
  o.learned = 0;
  o.mlp_blob = nullptr;
  o.flags = 0;
  o.diag = nullptr;
  const size_t rbytes = size_ratio_bytes(c.n, S);
  if (!o.workspace || o.workspace_bytes < rbytes) return CBP_E_NOMEM;
  o.workspace_bytes -= rbytes;
  double* rat = ratios ? ratios : (double*)((char*)o.workspace + o.workspace_bytes);
  const std::vector<frame_req> reqs = {
      frame_req{b1, b2, nullptr, b1->height - K1 + 1, b1->width - K1 + 1, nullptr, nullptr, nullptr}};
  std::vector<cbp_status> status;
  batch_build bb;
  const cbp_status s = build_batch(reqs, &o, kDefaultTuning, status, &bb, true);
  if (s != CBP_OK) return s;
  if (status[0] != CBP_OK) return status[0];
  // the probe's items: (candidate, pass, sample)
  const int items = c.n * 2 * S;
  int* starts = (int*)(bb.head.data() + head_desc_bytes(1));
  starts[Q_SIZE_PROBE * 2] = 0;
  starts[Q_SIZE_PROBE * 2 + 1] = items;
  chunk_view& cv = bb.chunks[0];
  cv.items[Q_SIZE_PROBE] = items;
  cv.grid[Q_SIZE_PROBE] = grid_for(items, 0);
  int nmax = 1;
  for (int i = 0; i < c.n; ++i) nmax = std::max(nmax, 2 * c.k1[i] - d);
  const int NL = 2 * (K1 + (K1 - d)) - 1;
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  const batch_ref br = {cv.descs, cv.starts, cv.nf, cv.ctr};
  hipStream_t st = (hipStream_t)opts->stream;
  std::lock_guard<std::mutex> lk(ds->launch_mu);
  (void)hipGetLastError();
  auto run = [&]() -> hipError_t {
    inline_head ih;
    const bool inl = make_inline_head(bb, &ih);
    if (!inl) CBP_TRY(upload_head(*ds, bb, st));
    if (b1->dtype == CBP_F32) {
      CBP_TRY(launch_fold<float>(br, cv.grid[Q_FOLD], 0, inl ? &ih : nullptr, st));
      CBP_TRY(launch_eval_rows<float>(br, cv.grid[Q_EVAL_ROWS], st));
    } else {
      CBP_TRY(launch_fold<double>(br, cv.grid[Q_FOLD], 0, inl ? &ih : nullptr, st));
      CBP_TRY(launch_eval_rows<double>(br, cv.grid[Q_EVAL_ROWS], st));
    }
    CBP_TRY(launch_eval_cols(br, cv.grid[Q_EVAL_COLS], st));
    CBP_TRY(launch_gram(br, cv.grid[Q_GRAM], st));
    CBP_TRY(launch_size_probe(br, cv.grid[Q_SIZE_PROBE], c, nmax, NL, rat, st));
    CBP_TRY(launch_size_decide(c, S, rat, result, st));
    return hipSuccess;
  };
  return run() == hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

// ------------------------------------------------------------------ the encoder and the 8-bit streams
cbp_status cbp_draw_kernel_pairs(uint64_t seed, int64_t frame0, int32_t nframes, int32_t k1, int32_t k2,
                                 int32_t samples, double* K1s, double* K2s, int32_t* attempts, double* min_ratio,
                                 void* stream) {
  if (!K1s || !K2s || !attempts || nframes < 1 || frame0 < 0) return CBP_E_INVALID;
  if (k1 < 1 || k2 < 1 || k1 > CBP_MAX_K || k2 > CBP_MAX_K) return CBP_E_SHAPE;
  const int S = samples ? samples : std::max(k1, k2);
  if (S < 1 || S > CBP_MAX_S) return CBP_E_INVALID;
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  (void)hipGetLastError();
  return note("launch_draw_pairs", launch_draw_pairs(seed, frame0, nframes, k1, k2, S, K1s, K2s, (int*)attempts,
                                                    min_ratio, (hipStream_t)stream)) == hipSuccess
             ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_encode(const cbp_image* latent, const double* K1, int32_t k1, const double* K2, int32_t k2,
                      cbp_image* b1, cbp_image* b2, void* stream) {
  if (!latent || !K1 || !K2 || !b1 || !b2) return CBP_E_INVALID;
  if (!valid_image(latent) || !valid_image(b1) || !valid_image(b2)) return CBP_E_INVALID;
  if (b1->dtype != latent->dtype || b2->dtype != latent->dtype || b1->channels != latent->channels ||
      b2->channels != latent->channels)
    return CBP_E_INVALID;
  if (k1 < 1 || k2 < 1 || k1 > CBP_MAX_K || k2 > CBP_MAX_K) return CBP_E_SHAPE;
  const int m = latent->height, n = latent->width;
  if (b1->height != m + k1 - 1 || b1->width != n + k1 - 1 || b2->height != m + k2 - 1 || b2->width != n + k2 - 1)
    return CBP_E_SHAPE;
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  (void)hipGetLastError();
  const int nch = latent->channels;
  const int64_t lcs = nch > 1 ? latent->channel_stride : 0, c1 = nch > 1 ? b1->channel_stride : 0,
                c2 = nch > 1 ? b2->channel_stride : 0;
  hipError_t e;
  if (latent->dtype == CBP_F32)
    e = launch_blur<float>((const float*)latent->data, latent->pitch, lcs, m, n, nch, K1, k1, K2, k2,
                           (float*)b1->data, b1->pitch, c1, (float*)b2->data, b2->pitch, c2, (hipStream_t)stream);
  else
    e = launch_blur<double>((const double*)latent->data, latent->pitch, lcs, m, n, nch, K1, k1, K2, k2,
                            (double*)b1->data, b1->pitch, c1, (double*)b2->data, b2->pitch, c2, (hipStream_t)stream);
  return note("launch_blur", e) == hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_quantize(const cbp_image* src, cbp_image* dst, int32_t drop_bits, void* stream) {
  if (!valid_image(src) || !valid_u8_image(dst) || drop_bits < 0 || drop_bits > 8) return CBP_E_INVALID;
  if (src->height != dst->height || src->width != dst->width || src->channels != dst->channels) return CBP_E_SHAPE;
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  (void)hipGetLastError();
  const int nch = src->channels;
  const int64_t scs = nch > 1 ? src->channel_stride : 0, dcs = nch > 1 ? dst->channel_stride : 0;
  hipError_t e;
  if (src->dtype == CBP_F32)
    e = launch_quantize<float>((const float*)src->data, src->pitch, scs, (unsigned char*)dst->data, dst->pitch, dcs,
                               src->height, src->width, nch, drop_bits, (hipStream_t)stream);
  else
    e = launch_quantize<double>((const double*)src->data, src->pitch, scs, (unsigned char*)dst->data, dst->pitch,
                                dcs, src->height, src->width, nch, drop_bits, (hipStream_t)stream);
  return note("launch_quantize", e) == hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_dequantize(const cbp_image* src, cbp_image* dst, void* stream) {
  if (!valid_u8_image(src) || !valid_image(dst)) return CBP_E_INVALID;
  if (src->height != dst->height || src->width != dst->width || src->channels != dst->channels) return CBP_E_SHAPE;
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  (void)hipGetLastError();
  const int nch = src->channels;
  const int64_t scs = nch > 1 ? src->channel_stride : 0, dcs = nch > 1 ? dst->channel_stride : 0;
  hipError_t e;
  if (dst->dtype == CBP_F32)
    e = launch_dequantize<float>((const unsigned char*)src->data, src->pitch, scs, (float*)dst->data, dst->pitch, dcs,
                                 src->height, src->width, nch, (hipStream_t)stream);
  else
    e = launch_dequantize<double>((const unsigned char*)src->data, src->pitch, scs, (double*)dst->data, dst->pitch,
                                  dcs, src->height, src->width, nch, (hipStream_t)stream);
  return note("launch_dequantize", e) == hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

const char* cbp_last_error(void) { return t_error; }

// ------------------------------------------------------------------ the learned form's network
int32_t cbp_mlp_param_count(void) { return MLP_NPARAM; }
size_t cbp_mlp_blob_size(void) { return sizeof(mlp_blob); }
size_t cbp_mlp_state_size(int32_t max_rows) { return max_rows >= 1 ? mlp_state_bytes(max_rows) : 0; }

cbp_status cbp_mlp_set_params(void* state, int32_t max_rows, const float* params, void* stream) {
  if (!state || !params || max_rows < 1) return CBP_E_INVALID;
  (void)hipGetLastError();
  return note("mlp_set_params", mlp_set_params(state, max_rows, params, (hipStream_t)stream)) == hipSuccess
             ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_mlp_get_params(const void* state, int32_t max_rows, float* params, void* stream) {
  if (!state || !params || max_rows < 1) return CBP_E_INVALID;
  return note("mlp_get_params", mlp_get_params(state, max_rows, params, (hipStream_t)stream)) == hipSuccess
             ? CBP_OK : CBP_E_DEVICE;
}

size_t cbp_mlp_checkpoint_size(void) { return (size_t)3 * MLP_NPARAM * sizeof(float); }

cbp_status cbp_mlp_save_state(const void* state, int32_t max_rows, float* out, void* stream) {
  if (!state || !out || max_rows < 1) return CBP_E_INVALID;
  (void)hipGetLastError();
  return note("mlp_save_state", mlp_save_state(state, max_rows, out, (hipStream_t)stream)) == hipSuccess
             ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_mlp_load_state(void* state, int32_t max_rows, const float* in, void* stream) {
  if (!state || !in || max_rows < 1) return CBP_E_INVALID;
  (void)hipGetLastError();
  return note("mlp_load_state", mlp_load_state(state, max_rows, in, (hipStream_t)stream)) == hipSuccess
             ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_mlp_gradients(void* state, int32_t max_rows, const float* X, const float* T, int32_t n,
                             float* loss, float* grads, void* stream) {
  if (!state || !X || !T || !loss || n < 1 || n > max_rows) return CBP_E_INVALID;
  (void)hipGetLastError();
  return note("mlp_gradients", mlp_gradients(state, max_rows, X, T, n, loss, grads, (hipStream_t)stream)) ==
                 hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_mlp_train_step(void* state, int32_t max_rows, const float* X, const float* T, int32_t n, float lr,
                              int32_t step, float* loss, void* stream) {
  if (!state || !X || !T || !loss || n < 1 || n > max_rows || step < 1 || !(lr > 0.0f)) return CBP_E_INVALID;
  (void)hipGetLastError();
  hipStream_t st = (hipStream_t)stream;
  if (note("mlp_gradients", mlp_gradients(state, max_rows, X, T, n, loss, nullptr, st)) != hipSuccess)
    return CBP_E_DEVICE;
  return note("mlp_adam_step", mlp_adam_step(state, max_rows, lr, step, st)) == hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_mlp_export(const void* state, int32_t max_rows, void* blob, void* stream) {
  if (!state || !blob || max_rows < 1) return CBP_E_INVALID;
  (void)hipGetLastError();
  return note("mlp_export", mlp_export(state, max_rows, blob, (hipStream_t)stream)) == hipSuccess ? CBP_OK
                                                                                              : CBP_E_DEVICE;
}

cbp_status cbp_mlp_forward(const void* blob, const float* X, int32_t n, float* out, void* stream) {
  if (!blob || !X || !out || n < 1) return CBP_E_INVALID;
  (void)hipGetLastError();
  return note("mlp_forward", mlp_forward_blob(blob, X, n, out, (hipStream_t)stream)) == hipSuccess ? CBP_OK
                                                                                                 : CBP_E_DEVICE;
}

cbp_status cbp_last_tuning(cbp_tuning* out) {
  if (!out) return CBP_E_INVALID;
  dev_state* ds = get_dev();
  if (!ds) return CBP_E_DEVICE;
  std::lock_guard<std::mutex> lk(ds->launch_mu);
  if (!ds->have_last) return CBP_E_INVALID;
  *out = ds->last;
  return CBP_OK;
}

void cbp_profile_enable(int32_t on) {
  profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.on = on != 0;
}

void cbp_profile_reset(void) {
  profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  for (int i = 0; i < PH_COUNT; ++i) { p.total[i] = 0.0; p.count[i] = 0; }
}

int32_t cbp_profile_read(double* ms_total, int64_t* counts, int32_t max_phases) {
  profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  for (const pending_pair& q : p.pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      p.total[q.phase] += ms;
      p.count[q.phase] += 1;
    }
    p.pool.push_back(q.a);
    p.pool.push_back(q.b);
  }
  p.pending.clear();
  for (int i = 0; i < PH_COUNT && i < max_phases; ++i) {
    if (ms_total) ms_total[i] = p.total[i];
    if (counts) counts[i] = p.count[i];
  }
  return PH_COUNT;
}

const char* cbp_profile_phase_name(int32_t phase) {
  if (phase < 0 || phase >= PH_COUNT) return "";
  return kPhaseNames[phase];
}

}  // extern "C"
