// C ABI of the CBP library (declared in include/cbp.h): host-side validation,
// frame plans and workspace layout, the launch chain, and phase timing.
//
// Every status returned here comes from host-side checks made before the
// first HIP call of the entry point, so invalid arguments never reach a
// kernel.  Launch failures are reported as CBP_E_DEVICE.
#include <mutex>
#include <vector>

#include "internal.h"

namespace cbp {

size_t finalize_lds_bytes(int S);
size_t sample_lds_bytes(int N);
size_t row_lds_bytes(int N, int esize);
size_t col_lds_bytes(int N, int cw, int esize);

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kLdsLimit = 160 * 1024;

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
  size_t fpart, ex, ey, corr, xvec, lam0, pq, cbuf, kern, t, u;
};

region_sizes regions(int Hmax, int Wmax, int kmax, int S, int nch, int esize) {
  region_sizes r;
  const int Px = smooth7(Wmax);
  const size_t hx = (size_t)Px / 2 + 1;
  const size_t ncf = 2 * (size_t)nch;
  r.fpart = ((size_t)(Hmax + 31) / 32 + 1) * ncf * S * (size_t)Wmax * sizeof(double);
  r.ex = ncf * S * (size_t)Wmax * sizeof(c64);
  r.ey = ncf * S * (size_t)Hmax * sizeof(c64);
  r.corr = 2 * (size_t)S * (4 * (size_t)kmax - 1) * sizeof(cdd);
  r.xvec = 2 * (size_t)S * 2 * kmax * sizeof(c64);
  r.lam0 = 2 * (size_t)S * sizeof(double);
  r.pq = 4 * (size_t)S * S * sizeof(c64);
  r.cbuf = (size_t)S * S * sizeof(cdd);
  r.kern = 2 * (size_t)CBP_MAX_K * CBP_MAX_K * sizeof(double);
  r.t = (size_t)nch * Hmax * hx * 2 * esize;
  r.u = (size_t)nch * Hmax * hx * 2 * esize;
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
  fp->off_lam0 = take(r.lam0);
  fp->off_pq = take(r.pq);
  fp->off_cbuf = take(r.cbuf);
  fp->off_kern = take(r.kern);
  fp->off_t1 = take(r.t);
  fp->off_t2 = take(r.t);
  fp->off_u = take(r.u);
  fp->total = o;
  return o;
}

int max_fft(int esize) { return esize == 4 ? CBP_MAX_FFT_F32 : CBP_MAX_FFT_F64; }

// Choose the column-pass strip width: as wide as LDS allows, but keep at
// least ~128 workgroups per channel when the spectrum is narrow.
int choose_cw(int Py, int hx, int esize) {
  int cw = 4;
  while (cw > 1 && (col_lds_bytes(Py, cw, esize) > kLdsLimit - 4096 || (hx + cw - 1) / cw < 128)) cw >>= 1;
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

cbp_status check_options(const cbp_options* o, int dtype) {
  if (!o) return CBP_E_INVALID;
  if (!(o->lambda >= 0.0) || o->tau != 0.0 || o->learned != 0 || o->flags != 0 || o->mlp_blob != nullptr)
    return o->learned != 0 || o->mlp_blob != nullptr ? CBP_E_UNSUPPORTED : CBP_E_INVALID;
  if (o->precision == CBP_PREC_FP64) return dtype == CBP_F64 ? CBP_OK : CBP_E_INVALID;
  if (o->precision == CBP_PREC_MIXED) return dtype == CBP_F32 ? CBP_OK : CBP_E_INVALID;
  if (o->precision == CBP_PREC_MFMA32 || o->precision == CBP_PREC_BF16) return CBP_E_UNSUPPORTED;
  return CBP_E_INVALID;
}

// Shapes -> plan.  All checks are host-side.
cbp_status make_plan(const cbp_image* b1, const cbp_image* b2, int m, int n, const cbp_options* o,
                     frame_plan* fp) {
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
  if (S < kmax || S > CBP_MAX_S) return CBP_E_INVALID;
  const int esize = b1->dtype == CBP_F32 ? 4 : 8;
  fp->H1 = b1->height; fp->W1 = b1->width; fp->H2 = b2->height; fp->W2 = b2->width;
  fp->Hmax = fp->H1 > fp->H2 ? fp->H1 : fp->H2;
  fp->Wmax = fp->W1 > fp->W2 ? fp->W1 : fp->W2;
  fp->m = m; fp->n = n; fp->k1 = k1; fp->k2 = k2; fp->S = S; fp->N = k1 + k2;
  fp->nch = b1->channels;
  fp->rpg = S * ((32 + S - 1) / S);
  fp->RG = (fp->Hmax + fp->rpg - 1) / fp->rpg;
  fp->Py = smooth7(fp->Hmax);
  fp->Px = smooth7(fp->Wmax);
  if (fp->Py > max_fft(esize) || fp->Px > max_fft(esize)) return CBP_E_SHAPE;
  if (!make_fft_plan(fp->Py, &fp->fy) || !make_fft_plan(fp->Px, &fp->fx)) return CBP_E_SHAPE;
  fp->hx = fp->Px / 2 + 1;
  fp->cw = choose_cw(fp->Py, fp->hx, esize);
  if (sample_lds_bytes(fp->N) > kLdsLimit || finalize_lds_bytes(S) > kLdsLimit ||
      row_lds_bytes(fp->Px, esize) > kLdsLimit || col_lds_bytes(fp->Py, fp->cw, esize) > kLdsLimit)
    return CBP_E_SHAPE;
  layout(fp, regions(fp->Hmax, fp->Wmax, kmax, S, fp->nch, esize));
  return CBP_OK;
}

template <typename T>
pair_view<T> view_of(const cbp_image* b1, const cbp_image* b2) {
  pair_view<T> v;
  v.b1 = (const T*)b1->data;
  v.b2 = (const T*)b2->data;
  v.p1 = b1->pitch; v.p2 = b2->pitch;
  v.cs1 = b1->channels > 1 ? b1->channel_stride : 0;
  v.cs2 = b2->channels > 1 ? b2->channel_stride : 0;
  v.H1 = b1->height; v.W1 = b1->width; v.H2 = b2->height; v.W2 = b2->width;
  v.nch = b1->channels;
  return v;
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

const char* kPhaseNames[PH_COUNT] = {"fold_cols", "eval_cols", "eval_rows", "gram", "sample_eig",
                                     "scale_assemble", "row_fft_fwd", "col_fft_filter", "row_fft_inv"};

// Side stream and fork/join events of one device (created once; default
// priority).  The row fold and the row FFT depend only on the input frames,
// so they run on the side stream beside the column fold -> Gram ->
// eigen-solve chain, which occupies few compute units.
struct fork_state {
  std::mutex launch_mu;   // one launch sequence at a time per device (the events are shared)
  bool ready = false;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_rows = nullptr, ev_fft = nullptr;
};

fork_state* get_fork() {
  static std::mutex mu;
  static fork_state states[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  fork_state& f = states[dev];
  if (!f.ready) {
    if (hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&f.ev_fork, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&f.ev_rows, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&f.ev_fft, hipEventDisableTiming) != hipSuccess) return nullptr;
    f.ready = true;
  }
  return &f;
}

template <typename T>
cbp_status run_frame(const cbp_image* b1, const cbp_image* b2, const frame_plan& fp, char* ws, double* K1,
                     double* K2, cbp_image* latent, const cbp_options* o, void* diag) {
  hipStream_t st = (hipStream_t)o->stream;
  const pair_view<T> v = view_of<T>(b1, b2);
  double* k1 = K1 ? K1 : (double*)(ws + fp.off_kern);
  double* k2 = K2 ? K2 : (double*)(ws + fp.off_kern) + CBP_MAX_K * CBP_MAX_K;
  fork_state* f = get_fork();
  if (!f) return CBP_E_DEVICE;
  std::lock_guard<std::mutex> launch_lock(f->launch_mu);
  hipStream_t side = f->side;
  // fork
  if (hipEventRecord(f->ev_fork, st) != hipSuccess) return CBP_E_DEVICE;
  if (hipStreamWaitEvent(side, f->ev_fork, 0) != hipSuccess) return CBP_E_DEVICE;
  if (launch_eval_rows<T>(v, fp, ws, side) != hipSuccess) return CBP_E_DEVICE;
  if (hipEventRecord(f->ev_rows, side) != hipSuccess) return CBP_E_DEVICE;
  if (latent && launch_row_fwd<T>(v, fp, ws, side) != hipSuccess) return CBP_E_DEVICE;
  if (hipEventRecord(f->ev_fft, side) != hipSuccess) return CBP_E_DEVICE;
  // main chain
  if (launch_eval_cols<T>(v, fp, ws, st) != hipSuccess) return CBP_E_DEVICE;
  if (hipStreamWaitEvent(st, f->ev_rows, 0) != hipSuccess) return CBP_E_DEVICE;
  if (launch_recover(fp, ws, k1, k2, diag, st) != hipSuccess) return CBP_E_DEVICE;
  // join (also when no latent is produced, so the side stream never runs ahead of the next call)
  if (hipStreamWaitEvent(st, f->ev_fft, 0) != hipSuccess) return CBP_E_DEVICE;
  if (latent) {
    const int64_t ocs = latent->channels > 1 ? latent->channel_stride : 0;
    if (launch_col_inv<T>(v, fp, ws, k1, k2, (T*)latent->data, latent->pitch, ocs, o->lambda, st) != hipSuccess)
      return CBP_E_DEVICE;
  }
  return CBP_OK;
}

cbp_status frame_call(const cbp_image* b1, const cbp_image* b2, cbp_image* latent, int m, int n, double* K1,
                      double* K2, const cbp_options* o, char* ws, size_t ws_bytes, void* diag) {
  frame_plan fp;
  const cbp_status s = make_plan(b1, b2, m, n, o, &fp);
  if (s != CBP_OK) return s;
  if (latent) {
    if (!valid_image(latent) || latent->dtype != b1->dtype || latent->channels != b1->channels) return CBP_E_INVALID;
  }
  if (!ws || ws_bytes < fp.total) return CBP_E_NOMEM;
  if (b1->dtype == CBP_F32) return run_frame<float>(b1, b2, fp, ws, K1, K2, latent, o, diag);
  return run_frame<double>(b1, b2, fp, ws, K1, K2, latent, o, diag);
}

}  // namespace

void prof_begin(int phase, hipStream_t st) {
  profiler& p = prof();
  if (!p.on) return;
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t e = p.get();
  if (!e) return;
  hipEventRecord(e, st);
  p.open[phase] = e;
}

void prof_end(int phase, hipStream_t st) {
  profiler& p = prof();
  if (!p.on) return;
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

const char* cbp_version(void) { return "0.1.0"; }

size_t cbp_diag_size(void) { return sizeof(cbp_diag); }

size_t cbp_workspace_size(int32_t maxH, int32_t maxW, int32_t maxk, int32_t channels, int32_t batch,
                          const cbp_options* opts) {
  if (maxH < 1 || maxW < 1 || maxk < 1 || maxk > CBP_MAX_K || channels < 1 || batch < 1) return 0;
  int S = maxk;
  int esize = 8;
  if (opts) {
    if (opts->samples > S) S = opts->samples;
    if (opts->precision == CBP_PREC_MIXED) esize = 4;
  }
  if (S > CBP_MAX_S) return 0;
  frame_plan fp;
  const size_t one = layout(&fp, regions(maxH, maxW, maxk, S, channels, esize));
  return one * (size_t)batch;
}

cbp_status cbp_eval_unit_circle(const cbp_image* b, int32_t S, double* ex, double* ey, const cbp_options* opts) {
  if (!valid_image(b) || !ex || !ey || !opts) return CBP_E_INVALID;
  if (S < 1 || S > CBP_MAX_S) return CBP_E_INVALID;
  const size_t need = ((size_t)(b->height + 31) / 32 + 1) * (size_t)S * b->width * sizeof(double);
  if (!opts->workspace || opts->workspace_bytes < need) return CBP_E_NOMEM;
  const hipError_t e = launch_eval_single(b->data, b->dtype, b->pitch, b->height, b->width, S,
                                          (char*)opts->workspace, ex, ey, (hipStream_t)opts->stream);
  return e == hipSuccess ? CBP_OK : CBP_E_DEVICE;
}

cbp_status cbp_recover_kernels(const cbp_image* b1, const cbp_image* b2, int32_t m, int32_t n, double* K1,
                               double* K2, const cbp_options* opts) {
  if (!K1 || !K2 || !opts) return CBP_E_INVALID;
  return frame_call(b1, b2, nullptr, m, n, K1, K2, opts, (char*)opts->workspace, opts->workspace_bytes,
                    opts->diag);
}

cbp_status cbp_deblur(const cbp_image* b1, const cbp_image* b2, cbp_image* latent, double* K1, double* K2,
                      const cbp_options* opts) {
  if (!opts || !latent) return CBP_E_INVALID;
  return frame_call(b1, b2, latent, latent->height, latent->width, K1, K2, opts, (char*)opts->workspace,
                    opts->workspace_bytes, opts->diag);
}

cbp_status cbp_deblur_batch(int32_t nframes, const cbp_image* b1s, const cbp_image* b2s, cbp_image* latents,
                            double* const* K1s, double* const* K2s, cbp_status* per_frame, const cbp_options* opts) {
  if (nframes < 1 || !b1s || !b2s || !latents || !opts) return CBP_E_INVALID;
  const size_t slice = (opts->workspace_bytes / (size_t)nframes) & ~(kAlign - 1);
  cbp_status first = CBP_OK;
  for (int f = 0; f < nframes; ++f) {
    char* ws = opts->workspace ? (char*)opts->workspace + (size_t)f * slice : nullptr;
    void* diag = opts->diag ? (void*)((cbp_diag*)opts->diag + f) : nullptr;
    const cbp_status s = frame_call(&b1s[f], &b2s[f], &latents[f], latents[f].height, latents[f].width,
                                    K1s ? K1s[f] : nullptr, K2s ? K2s[f] : nullptr, opts, ws, slice, diag);
    if (per_frame) per_frame[f] = s;
    if (s != CBP_OK && first == CBP_OK) first = s;
  }
  return first;
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
