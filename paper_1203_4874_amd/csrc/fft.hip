// Two-channel regularised Fourier division (Sec. 4: the latent is obtained by
// dividing a blurred frame by the recovered kernel in the Fourier domain;
// Sec. 5: an inverse FFT of the divided spectrum).  Over a Py x Px grid that
// covers both frames (no wrap-around of the full convolutions):
//   Lhat = (conj(K1hat) B1hat + conj(K2hat) B2hat) / (|K1hat|^2 + |K2hat|^2 + lambda),
//   L    = IFFT2(Lhat) cropped to m x n
// (with the single-channel variant, the paper's B1 / K1: the K2 terms drop).
//
// Three passes, each a hand-written Stockham FFT in LDS (fft_core.h):
//   1. row pass: row y of B1 and row y of B2 packed as one complex row
//      B1 + i B2, one complex FFT, split into the two half spectra
//      T_c[y][0..Px/2] (Hermitian symmetry of real rows);
//   2. column pass: for a strip of half-spectrum columns, forward FFT of the
//      T_1 and T_2 columns (zero rows beyond H_c), the filter above with the
//      kernel spectra evaluated in place from the k x k kernels, inverse FFT,
//      keep the first m rows -> U[y][kx];
// T and U rows have a pitch of hxp >= hx entries, a multiple of 128 bytes, so
// the column pass reads and writes whole row segments.
//   3. inverse row pass: two rows of U packed as one complex spectrum (each
//      completed by Hermitian symmetry), one inverse FFT, real / imaginary
//      parts are the two output rows, scaled by 1/(Py Px), cropped to n.
// T is float (mixed form) or double (FP64 form).
#include <algorithm>
#include <atomic>
#include "eigsmall.h"
#include "internal.h"

namespace cbp {

namespace {

// ---------------------------------------------------------------- in-place passes
// The transforms run in place in LDS: every pass reads its butterflies'
// inputs into registers, synchronises, and writes the outputs over them (one
// buffer instead of a ping-pong pair).  Twiddles come from the plan's pass
// tables in LDS (fft_core.h tw_pitch), FP64 sincospi rounded once to T (one
// read per twiddle).

// threadIdx.x behind an empty asm statement: values derived from it are
// recomputed where they are used instead of being hoisted out of the item
// loop, where they would stay live (one register each) across the kernel.
__device__ __attribute__((always_inline)) inline int local_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Butterflies per thread of a radix-R pass over at most MAXE entries.
template <int NT, int R, int MAXE>
constexpr int ip_mb() { return (MAXE / R + NT - 1) / NT; }

// w_N^t, t < N, into tw when the table holds another length (tabN: the
// length it holds, wave-uniform); the caller synchronises before use.
template <typename T>
__device__ __attribute__((always_inline)) inline void full_twiddles(cplx<T>* tw, int N, int& tabN) {
  if (tabN == N) return;
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * (double)t / (double)N, &sn, &cs);
    tw[t] = {T(cs), T(sn)};
  }
  tabN = N;
}

// The pass twiddle tables of plan p into tws when they hold another plan's
// (tabN, tabCode: the length and pass order they hold, wave-uniform); the
// caller synchronises before use.  Entry k P + r - 1 of the pass with stride
// Ns is w_(Ns R)^(r k): the angle r k / (Ns R) equals r k (N / (Ns R)) / N
// exactly in FP64, so the values are those of the full table w_N^t.
template <typename T>
__device__ __attribute__((always_inline)) inline void pass_twiddles(cplx<T>* tws, const fft_plan& p, int& tabN,
                                                                    unsigned long long& tabCode) {
  if (tabN == p.N && tabCode == p.code) return;
  int Ns = 1, off = 0;
  for (int s = 0; s < p.npass; ++s) {
    const int R = plan_radix(p, s);
    if (Ns > 1) {
      const int P = tw_pitch(R), n = Ns * P;
      for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int k = e / P, r = e - k * P + 1;
        double sn = 0.0, cs = 1.0;
        if (r < R) sincospi(-2.0 * (double)(r * k) / (double)(Ns * R), &sn, &cs);
        tws[off + e] = {T(cs), T(sn)};
      }
      off += n;
    }
    Ns *= R;
  }
  tabN = p.N;
  tabCode = p.code;
}

// One radix-R pass (stride Ns) over ncol transforms of length N at
// buf + c ld, in place: butterfly j of transform c reads
// buf[c ld + j + r N/R] and writes buf[c ld + (j - k) R + k + r Ns],
// k = j mod Ns (the Stockham indexing of fft_core.h, read and write phases
// separated by a barrier); tws: the pass's twiddle table.  ncol (a power of
// two) N <= MAXE.  Butterfly b of the pass is (c, j) = (b mod ncol,
// b / ncol): consecutive lanes take the same j of consecutive transforms,
// whose entries the strip's column stride puts in distinct banks.
template <int R, int DIR, int NT, int MAXE, typename T>
__device__ __attribute__((always_inline)) inline void ip_pass(cplx<T>* buf, int ld, int N, int Ns,
                                                              const cplx<T>* tws, int ncol) {
  constexpr int MB = ip_mb<NT, R, MAXE>();
  const int NR = N / R;
  const int total = NR * ncol;
  const int lnc = __builtin_ctz(ncol);
  const float rns = 1.0f / (float)Ns;
  cplx<T> v[MB][R];
  int pos[MB];
  const int tid = local_tid();
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int b = tid + q * NT;
    pos[q] = -1;
    if (b < total) {
      const int c = b & (ncol - 1), j = b >> lnc;
      const int k = Ns > 1 ? j - mul24(fdiv_floor(j, rns), Ns) : 0;
      const cplx<T>* src = buf + mul24(c, ld);
      const int base = Ns > 1 ? stockham_read<R, DIR, true>(src, NR, tws, j, k, v[q])
                              : stockham_read<R, DIR, false>(src, NR, tws, j, k, v[q]);
      pos[q] = mul24(c, ld) + base;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MB; ++q)
    if (pos[q] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pos[q] + mul24(r, Ns)] = v[q][r];
    }
  __syncthreads();
}

// All passes of plan p over ncol transforms (ncol p.N <= MAXE), in place;
// tws: the plan's pass tables (pass_twiddles).  R9: the plan may hold
// radix-9 passes (the row plans; the column plans do not, which keeps the
// column pass's registers at the radix-8 pass).
template <int DIR, int NT, int MAXE, bool R9 = false, typename T>
__device__ __attribute__((always_inline)) inline void ip_fft(cplx<T>* buf, int ld, const fft_plan& p,
                                                             const cplx<T>* tws, int ncol) {
  int Ns = 1;
  const cplx<T>* t = tws;   // this pass's table (the first pass, Ns = 1, has none)
  for (int s = 0; s < p.npass; ++s) {
    const int R = plan_radix(p, s);
    if constexpr (R9) {
      if (R == 9) {
        ip_pass<9, DIR, NT, MAXE>(buf, ld, p.N, Ns, t, ncol);
        if (Ns > 1) t += Ns * tw_pitch(9);
        Ns *= 9;
        continue;
      }
    }
    switch (R) {
      case 2: ip_pass<2, DIR, NT, MAXE>(buf, ld, p.N, Ns, t, ncol); break;
      case 3: ip_pass<3, DIR, NT, MAXE>(buf, ld, p.N, Ns, t, ncol); break;
      case 4: ip_pass<4, DIR, NT, MAXE>(buf, ld, p.N, Ns, t, ncol); break;
      case 5: ip_pass<5, DIR, NT, MAXE>(buf, ld, p.N, Ns, t, ncol); break;
      case 7: ip_pass<7, DIR, NT, MAXE>(buf, ld, p.N, Ns, t, ncol); break;
      default: ip_pass<8, DIR, NT, MAXE>(buf, ld, p.N, Ns, t, ncol); break;
    }
    if (Ns > 1) t += Ns * tw_pitch(R);
    Ns *= R;
  }
}

// Largest row length (entries) of the row passes.
constexpr int ROW_MAXE = CBP_MAX_FFT_F32 > CBP_MAX_FFT_F64 ? CBP_MAX_FFT_F32 : CBP_MAX_FFT_F64;

// ---------------------------------------------------------------- pass 1
// Items: (channel, row group g, residue r): the rows y = g rpg + r + S i,
// i < rpg / S, y < Hmax, in increasing y.  Each row of both frames is packed
// as B1 + i B2 and transformed; while the rows pass, the workgroup folds them
// (the column fold of k_fold_cols: the same rows of the same residue and
// group, summed in increasing y in FP64, hence the same bits) and writes
// the group's partial sums, so the frames are read once.  With with_ey, the
// unit-circle evaluation of both rows (fold modulo S and S-point DFT, as
// k_eval_rows: the same lanes, the same order, hence the same bits) is taken
// from the row in LDS; waves 0-1 fold frame (w & 1).  The grid is
// persistent: a workgroup loads its next row into registers while it
// transforms the current one.
static_assert(CBP_MAX_FFT_F32 <= 8 * 256 && CBP_MAX_FFT_F64 <= 8 * 256, "one row is eight loads per thread");

template <typename T>
__global__ __launch_bounds__(256) void k_row_fwd(batch_ref br, int with_ey) {
  extern __shared__ __attribute__((aligned(16))) char sm_rf[];
  __shared__ double gy[2][CBP_MAX_S];
  __shared__ double fpart_l[2][128];
  __shared__ c64 twS[CBP_MAX_S];
  __shared__ int st[BATCH_CHUNK + 1];
  const int nf = br.nframes;
  const int* sq = br.starts + (size_t)Q_ROW_FWD * (nf + 1);
  for (int t = threadIdx.x; t <= nf; t += blockDim.x) st[t] = sq[t];
  __syncthreads();
  int first, end, step;
  xcd_items(__builtin_amdgcn_readfirstlane(st[nf]), (int)blockIdx.x, (int)gridDim.x, first, end, step);
  // frame of item it (st[fi] <= it < st[fi + 1]), wave-uniform
  auto frame_of = [&](int it) __attribute__((always_inline)) {
    int lo = 0, hi = nf;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (st[mid] <= it) lo = mid;
      else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
  };
  // descriptors are read-only while kernels run: reading them through the
  // constant address space with a wave-uniform index lets the scalar unit
  // load them into SGPRs
  auto desc = [&](int fi) __attribute__((always_inline)) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) frame_desc cdesc;
    return ((const cdesc*)br.descs)[fi];
#else
    return br.descs[fi];
#endif
  };
  // item it -> (channel, first row y0, rows of the item below Hmax)
  struct rows_of_item { int ch, g, r, y0, nv; };
  auto item_rows = [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int S = d.S, RG = d.RG, gi = d.rpg / S;
    rows_of_item q;
    q.r = item % S;
    const int rest = item / S;
    q.g = rest % RG;
    q.ch = rest / RG;
    q.y0 = q.g * d.rpg + q.r;
    q.nv = q.y0 >= d.Hmax ? 0 : min(gi, (d.Hmax - 1 - q.y0) / S + 1);
    return q;
  };
  // the two rows y of channel ch into registers: eight loads per frame and
  // thread, from clamped (always valid) addresses; entries outside the frame
  // are zeroed when they are used
  T uv[8], wv[8];
  auto fetch = [&](const frame_desc& d, int ch, int y) __attribute__((always_inline)) {
    // row pointers clamped to each frame's last row (rows past it read as zero)
    const T* r1 = (const T*)d.b1 + ch * d.cs1 + (int64_t)min(y, d.H1 - 1) * d.p1;
    const T* r2 = (const T*)d.b2 + ch * d.cs2 + (int64_t)min(y, d.H2 - 1) * d.p2;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int x = t * 256 + local_tid();
      uv[t] = r1[min(x, d.W1 - 1)];
      wv[t] = r2[min(x, d.W2 - 1)];
    }
  };
  // the first row of the first item at or after it that has rows (it >= end: none)
  auto fetch_from = [&](int it) __attribute__((always_inline)) {
    for (; it < end; it += step) {
      const int fi = frame_of(it);
      const frame_desc d = desc(fi);
      const rows_of_item q = item_rows(d, it - __builtin_amdgcn_readfirstlane(st[fi]));
      if (q.nv > 0) {
        fetch(d, q.ch, q.y0);
        return;
      }
    }
  };
  fetch_from(first);
  int tabN = 0;                  // plan of the pass tables in LDS (length,
  unsigned long long tabCode = 0;  // pass order)
  int tabS = 0;                  // S of the unit twiddles in twS
  for (int it = first; it < end; it += step) {
    const int fi = frame_of(it);
    const frame_desc d = desc(fi);
    const rows_of_item q = item_rows(d, it - __builtin_amdgcn_readfirstlane(st[fi]));
    const fft_plan& px = d.fx;
    const int N = px.N, hx = d.hx, S = d.S;
    cplx<T>* a = (cplx<T>*)sm_rf;
    cplx<T>* twf = a + N;
    const int ch = q.ch;
    const int W1 = d.W1, W2 = d.W2;
    // the column fold of this item's rows, both frames (FP64, increasing y)
    double f1[8], f2[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) f1[t] = f2[t] = 0.0;
    for (int i = 0; i < q.nv; ++i) {
      const int y = q.y0 + S * i;
      const bool in1 = y < d.H1, in2 = y < d.H2;
      pass_twiddles(twf, px, tabN, tabCode);
      if (with_ey && S != tabS) {
        // w_t for the row evaluation (made again only when S changes; the
        // barrier after the row's store orders it before its use)
        unit_twiddles(twS, S);
        tabS = S;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int x = t * 256 + local_tid();
        const T u1 = (in1 && x < W1) ? uv[t] : T(0), u2 = (in2 && x < W2) ? wv[t] : T(0);
        f1[t] += (double)u1;
        f2[t] += (double)u2;
        if (x < N) a[x] = {u1, u2};
      }
      __syncthreads();
      // the next row is in flight while this one is transformed
      if (i + 1 < q.nv) fetch(d, ch, y + S);
      else fetch_from(it + step);
      if (with_ey) {
        // the row evaluation of both rows (k_eval_rows's lanes and order):
        // waves 2 fr, 2 fr + 1 fold frame fr's row into partials, lane
        // g S + r of the pair summing x = r + S (g + G i); the residues then
        // add their G partials in order
        const int G = 128 / S;
        const int fr = threadIdx.x >> 7, l = threadIdx.x & 127;
        const int gl = l / S, rr0 = l - gl * S;
        const bool inr = fr ? in2 : in1;
        {
          double acc = 0.0;
          if (inr && gl < G) acc = fold_strided((const T*)a + fr, 2, rr0 + S * gl, S * G, fr ? W2 : W1);
          fpart_l[fr][l] = acc;
        }
        __syncthreads();
        if (l < S) {
          double sr = fpart_l[fr][l];
          for (int gq = 1; gq < G; ++gq) sr += fpart_l[fr][gq * S + l];
          gy[fr][l] = sr;
        }
        __syncthreads();
        if (l < S && inr) d.ey[((size_t)(2 * ch + fr) * S + l) * d.Hmax + y] = dft_at(gy[fr], 1, twS, S, l);
      }
      ip_fft<-1, 256, ROW_MAXE, true>(a, N, px, twf, 1);
      const cplx<T>* z = a;
      cplx<T>* o1 = (cplx<T>*)d.t1 + (int64_t)ch * d.Hmax * d.hxp + (int64_t)y * d.hxp;
      cplx<T>* o2 = (cplx<T>*)d.t2 + (int64_t)ch * d.Hmax * d.hxp + (int64_t)y * d.hxp;
      for (int k = threadIdx.x; k < hx; k += blockDim.x) {
        const cplx<T> zk = z[k];
        const cplx<T> zn = conj(z[k == 0 ? 0 : N - k]);
        const cplx<T> s = zk + zn, df = zk - zn;
        if (in1) o1[k] = {T(0.5) * s.re, T(0.5) * s.im};       // (Z_k + conj Z_{N-k}) / 2
        if (in2) o2[k] = {T(0.5) * df.im, T(-0.5) * df.re};    // (Z_k - conj Z_{N-k}) / (2i)
      }
      __syncthreads();
    }
    // the group's column-fold partials (k_fold_cols's layout), for x < W
    double* fp1 = d.fpart + (((size_t)q.g * d.ncf + 2 * ch) * S + q.r) * (size_t)d.Wmax;
    double* fp2 = d.fpart + (((size_t)q.g * d.ncf + 2 * ch + 1) * S + q.r) * (size_t)d.Wmax;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int x = t * 256 + local_tid();
      if (x < W1) fp1[x] = f1[t];
      if (x < W2) fp2[x] = f2[t];
    }
  }
}

// ---------------------------------------------------------------- pass 2
// The column pass keeps one strip of cw columns (cw up to 16: up to 128-byte
// row segments of T) in LDS, column-major with an odd leading dimension, and
// transforms it in place.  One buffer per strip instead of two frames'
// ping-pong pairs is what makes wide strips fit; frame 2's spectrum waits in
// registers while frame 1 is transformed.  The workgroup has NT = 512 or 1024
// threads.

// Column stride of a strip in LDS: the smallest ld >= N whose residue modulo
// the entries of one 128-byte bank row (16 FP32 / 8 FP64 complex) is that
// count over cw (1 when cw is larger).  The row segments the strip is loaded
// from and stored to (cw columns of consecutive rows on consecutive lanes)
// then fall in distinct banks.
template <typename T>
__host__ __device__ inline int col_ld(int N, int cw) {
  constexpr int B = 128 / (int)sizeof(cplx<T>);
  const int t = cw < B ? B / cw : 1;
  return N + (((t - N) % B) + B) % B;
}

// Largest cw * N of a strip: 9 FP32 (4.5 FP64) complex entries per thread,
// so each thread's share of a pass and of the stashed spectrum stays in
// registers.
template <typename T, int NT>
constexpr int col_max_elems() { return NT * 72 / (int)sizeof(cplx<T>); }


// The strip's entries as each thread holds them for the stash and the
// filter: column c = tid / (NT / cw) (wave-uniform: NT / cw >= 64) and rows in
// groups of g = 4, 2 or 1 (g divides N): rows y + j N/g, j < g,
// y = tid mod (NT / cw) + i NT / cw < N/g, whose twiddles w_N^(y + j N/g)
// differ by the g-th roots of unity.  Group i holds slots g i .. g i + g - 1.
template <typename T, int NT, int G>
constexpr int col_groups() { return (col_max_elems<T, NT>() / G + NT - 1) / NT; }

// Items: (strip of cw columns, channel).  A workgroup that owns several
// items loads the next strip (and frame 1's strip of the current item) into
// registers while it transforms.
// G: rows per group of the filter's kernel-spectrum evaluation.  A launch
// takes the items of the frames whose group (col_group_size of their N) is
// G and passes over the others, which a launch with their G takes: each
// frame is filtered with its own group whatever the batch, and a
// compile-time group keeps the stashed spectrum's slots compile-time
// indices, in registers.
template <typename T, int NT, int G>
__global__ __launch_bounds__(NT, sizeof(T) == 4 ? 4 : 2) void k_col_filter(batch_ref br) {
  extern __shared__ __attribute__((aligned(16))) char sm_cf[];
  __shared__ int st[BATCH_CHUNK + 1];
  constexpr int SM = G * col_groups<T, NT, G>();
  constexpr int PF = (col_max_elems<T, NT>() + NT - 1) / NT;   // strip entries per thread
  constexpr int LNT = NT == 1024 ? 10 : NT == 512 ? 9 : 8;
  __shared__ int s_next[2];   // the workgroup's next items (thread 0 takes them), alternate slots
  const int nf = br.nframes;
  const int* sq = br.starts + (size_t)Q_COL * (nf + 1);
  for (int t = threadIdx.x; t <= nf; t += NT) st[t] = sq[t];
  __syncthreads();
  // items handed out dynamically from this group's counters (dyn_items);
  // with no more items than workgroups, one item per workgroup as
  // xcd_items assigns them (a workgroup that took two, one ahead, would
  // leave another idle)
  const int ntot = __builtin_amdgcn_readfirstlane(st[nf]);
  const bool dyn = ntot > (int)gridDim.x;
  const dyn_items q = make_dyn_items(br.ctr + CTR_COL + 8 * (G == 4 ? 0 : G == 2 ? 1 : 2), ntot, (int)blockIdx.x,
                                     (int)gridDim.x);
  const int end = q.hi;
  auto frame_of = [&](int it) __attribute__((always_inline)) {
    int lo = 0, hi = nf;   // st[lo] <= it < st[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (st[mid] <= it) lo = mid;
      else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
  };
  auto desc = [&](int fi) __attribute__((always_inline)) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) frame_desc cdesc;
    return ((const cdesc*)br.descs)[fi];
#else
    return br.descs[fi];
#endif
  };
  // strip entries e = y cw + c (cw consecutive threads read one row
  // segment) of frame fr of item it into registers, from clamped (always
  // valid) addresses; rows past the frame and columns past hx are zeroed when
  // they are stored to LDS
  cplx<T> pre[PF];
  auto fetch = [&](int it, int fr) __attribute__((always_inline)) {
    const int fi = frame_of(it);
    const frame_desc d = desc(fi);
    const int item = it - __builtin_amdgcn_readfirstlane(st[fi]);
    const int cw = d.cw, hx = d.hx, tp = d.hxp, lcw = __builtin_ctz(cw);
    const int nstrip = (hx + cw - 1) / cw;
    const int kx0 = (item % nstrip) * cw, ch = item / nstrip;
    const int Hf = fr ? d.H2 : d.H1;
    const cplx<T>* src = (const cplx<T>*)(fr ? d.t2 : d.t1) + ch * (int64_t)d.Hmax * tp;
    const int tid = local_tid();
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * NT;
      const int y = e >> lcw, c = e & (cw - 1);
      pre[i] = src[(int64_t)min(y, Hf - 1) * tp + min(kx0 + c, hx - 1)];
    }
  };
  auto first_frame = [&](int it) __attribute__((always_inline)) {
    return (desc(frame_of(it)).variant & VAR_DIVIDE_B1) ? 0 : 1;   // frame 2 first when both are divided
  };
  // Thread 0: from the item raw taken (its counter value, whose atomic may
  // still be in flight), the first item of a frame with group G (end: none;
  // the items of other groups are passed over, their launch has its own
  // counters).
  auto settle = [&](int raw) __attribute__((always_inline)) {
    int i = raw;
    while (i < end && col_group_size(desc(frame_of(i)).fy.N) != G) i = dyn ? q.take() : end;
    return i;
  };
  // one item ahead: the counter value taken while an item is processed is
  // read only when the next one starts, so the atomic's latency is hidden
  int ahead = end;
  if (threadIdx.x == 0) {
    if (dyn) {
      s_next[0] = settle(q.take());
      ahead = q.lo + atomicAdd(q.ctr, 1);
    } else {
      int first, last, step;
      xcd_items(ntot, (int)blockIdx.x, (int)gridDim.x, first, last, step);
      s_next[0] = settle(first < last ? first : end);
    }
  }
  __syncthreads();
  const int it0 = __builtin_amdgcn_readfirstlane(s_next[0]);
  if (it0 < end) fetch(it0, first_frame(it0));
  int tabN = 0;                   // length of the full twiddle table in LDS
  int tabNp = 0;                  // plan of the pass tables in LDS (length,
  unsigned long long tabCode = 0;   // pass order)
  for (int it = it0, nit, par = 1; it < end; it = nit, par ^= 1) {
    // the item after this one, read by every thread after the next barrier
    // (slot par: its last reads were two items ago)
    if (threadIdx.x == 0) {
      s_next[par] = settle(ahead < end ? ahead : end);
      ahead = dyn ? q.lo + atomicAdd(q.ctr, 1) : end;
    }
    const int fi = frame_of(it);
    const frame_desc d = desc(fi);
    const int item = it - __builtin_amdgcn_readfirstlane(st[fi]);
    const fft_plan& py = d.fy;
    const int N = py.N, cw = d.cw, hx = d.hx, tp = d.hxp, m = d.m;
    const int ld = col_ld<T>(N, cw);
    const int k1 = d.k1, k2 = d.k2, H1 = d.H1, H2 = d.H2;
    const T lam = (T)d.lambda;
    const bool two = !(d.variant & VAR_DIVIDE_B1);   // two-channel division, or B1 / K1 alone
    cplx<T>* buf = (cplx<T>*)sm_cf;                   // [cw][ld]
    cplx<T>* kr = buf + (size_t)cw * ld;              // [cw][2][CBP_MAX_K] row DFTs of the kernels at kx
    cplx<T>* tw = kr + (size_t)cw * 2 * CBP_MAX_K;    // [N] w_N^t (the filter's kernel spectra)
    // the filter's row groups (see col_groups) and its w_N^(G y), y < N / G
    cplx<T>* twg = tw + N;
    cplx<T>* twp = G > 1 ? twg + N / G : twg;         // the plan's pass tables
    const int nstrip = (hx + cw - 1) / cw;
    const int kx0 = (item % nstrip) * cw, ch = item / nstrip;
    const int lcw = __builtin_ctz(cw);                // cw is a power of two
    const int tot = N << lcw;
    // the registers' strip into buf[c ld + y]
    auto spill = [&](int Hf) __attribute__((always_inline)) {
      const int tid = local_tid();
#pragma unroll
      for (int i = 0; i < PF; ++i) {
        const int e = tid + i * NT;
        const int y = e >> lcw, c = e & (cw - 1);
        if (e < tot) buf[mul24(c, ld) + y] = (y < Hf && kx0 + c < hx) ? pre[i] : cplx<T>{T(0), T(0)};
      }
    };
    if (G > 1 && tabN != N)
      for (int y = threadIdx.x; y < N / G; y += NT) {
        double sn, cs;
        sincospi(-2.0 * (double)(G * y) / (double)N, &sn, &cs);   // = w_N^t, t = G y, as full_twiddles
        twg[y] = {T(cs), T(sn)};
      }
    full_twiddles(tw, N, tabN);
    pass_twiddles(twp, py, tabNp, tabCode);
    // the kernels' row DFTs at this strip's columns (k_kernel_dft), zero past hx
    {
      const cplx<T>* krg = (const cplx<T>*)d.kr;
      for (int e = threadIdx.x; e < cw * 2 * CBP_MAX_K; e += NT) {
        const int c = e / (2 * CBP_MAX_K);
        kr[e] = kx0 + c < hx ? krg[(size_t)kx0 * 2 * CBP_MAX_K + e] : cplx<T>{T(0), T(0)};
      }
    }
    // the entries this thread holds (see col_groups): f(group size, slot of
    // the group's first row, column, y, N / group size)
    auto for_held = [&](auto&& f) __attribute__((always_inline)) {
      const int tid = local_tid();
      const int ltpc = LNT - lcw;
      const int c = tid >> ltpc, r = tid & ((1 << ltpc) - 1);
      const int q = N / G;
#pragma unroll
      for (int i = 0; i < col_groups<T, NT, G>(); ++i) {
        const int y = r + (i << ltpc);
        if (y < q) f(std::integral_constant<int, G>(), G * i, c, y, q);
      }
    };
    cplx<T> st2[SM];
    if (two) {
      spill(H2);
      __syncthreads();
      fetch(it, 0);   // frame 1's strip in flight while frame 2's is transformed
      ip_fft<-1, NT, col_max_elems<T, NT>()>(buf, ld, py, twp, cw);
      for_held([&](auto GC, int a, int c, int y, int q) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < GC(); ++j) st2[a + j] = buf[mul24(c, ld) + y + j * q];
      });
      __syncthreads();   // buf is refilled with frame 1
    }
    spill(H1);
    __syncthreads();
    // the next item's first strip in flight while this one is finished
    nit = __builtin_amdgcn_readfirstlane(s_next[par]);
    if (nit < end) fetch(nit, first_frame(nit));
    ip_fft<-1, NT, col_max_elems<T, NT>()>(buf, ld, py, twp, cw);
    // filter: the combined spectrum in place of frame 1's
    const int kmax = k1 > k2 ? k1 : k2;
    auto filt = [&](cplx<T>* at, const cplx<T>& kh1, const cplx<T>& kh2, const cplx<T>& b2)
        __attribute__((always_inline)) {
      const cplx<T> B1 = *at;
      const cplx<T> num = two ? cmulc(kh1, B1) + cmulc(kh2, b2) : cmulc(kh1, B1);
      const T kk = two ? norm2(kh1) + norm2(kh2) : norm2(kh1);
      const T den = kk + lam;
      const T inv = den > T(0) ? T(1) / den : T(0);
      // where both kernel spectra vanish (a zeroed kernel pair) the
      // quotient is zero, whatever the frames hold
      *at = kk > T(0) ? cplx<T>{num.re * inv, num.im * inv} : cplx<T>{T(0), T(0)};
    };
    for_held([&](auto GC, int a, int c, int y, int q) __attribute__((always_inline)) {
      // kernel spectra at (ky, kx) = sum_yy kr[yy] z^yy, z = w_N^ky.  For the
      // group's rows ky = y + j N/g (z = w_N^y times the g-th roots of unity
      // (-i)^(4j/g)): K = sum_p z^p E_p(z^g), E_p(u) = sum_t kr[g t + p] u^t
      // by Horner's rule in u = w_N^(g y), then the g-point DFT of the
      // z^p E_p.  kr is zero beyond each kernel's size; the column is
      // wave-uniform.
      constexpr int g = GC();
      const cplx<T>* kr1 = kr + (size_t)c * 2 * CBP_MAX_K;
      const cplx<T>* kr2 = kr1 + CBP_MAX_K;
      const int nt = (kmax + g - 1) / g;          // coefficients per E_p
      const cplx<T> u = g == 1 ? tw[y] : twg[y];
      cplx<T> P1[g], P2[g];
#pragma unroll
      for (int p = 0; p < g; ++p) {
        const int top = g * (nt - 1) + p;
        cplx<T> e1 = top < CBP_MAX_K ? kr1[top] : cplx<T>{T(0), T(0)};
        cplx<T> e2 = top < CBP_MAX_K ? kr2[top] : cplx<T>{T(0), T(0)};
        for (int t = nt - 2; t >= 0; --t) {
          e1 = e1 * u + kr1[g * t + p];
          e2 = e2 * u + kr2[g * t + p];
        }
        if (p > 0) {
          const cplx<T> zp = tw[p * y];
          e1 = zp * e1;
          e2 = zp * e2;
        }
        P1[p] = e1;
        P2[p] = e2;
      }
      cplx<T>* col = buf + mul24(c, ld) + y;
      if constexpr (g == 1) {
        filt(col, P1[0], P2[0], st2[a]);
      } else if constexpr (g == 2) {
        filt(col, P1[0] + P1[1], P2[0] + P2[1], st2[a]);
        filt(col + q, P1[0] - P1[1], P2[0] - P2[1], st2[a + 1]);
      } else {
        // rows y, y + N/4, y + N/2, y + 3N/4: roots 1, -i, -1, i
        const cplx<T> s02_1 = P1[0] + P1[2], d02_1 = P1[0] - P1[2], s13_1 = P1[1] + P1[3], d13_1 = P1[1] - P1[3];
        const cplx<T> s02_2 = P2[0] + P2[2], d02_2 = P2[0] - P2[2], s13_2 = P2[1] + P2[3], d13_2 = P2[1] - P2[3];
        const cplx<T> md13_1 = mul_i(d13_1, -1), md13_2 = mul_i(d13_2, -1);   // -i (P1 - P3)
        filt(col, s02_1 + s13_1, s02_2 + s13_2, st2[a]);
        filt(col + q, d02_1 + md13_1, d02_2 + md13_2, st2[a + 1]);
        filt(col + 2 * q, s02_1 - s13_1, s02_2 - s13_2, st2[a + 2]);
        filt(col + 3 * q, d02_1 - md13_1, d02_2 - md13_2, st2[a + 3]);
      }
    });
    __syncthreads();
    ip_fft<+1, NT, col_max_elems<T, NT>()>(buf, ld, py, twp, cw);
    // the first m rows, row segments of cw columns
    cplx<T>* uo = (cplx<T>*)d.u + (int64_t)ch * m * tp;
    for (int e = threadIdx.x; e < (m << lcw); e += NT) {
      const int y = e >> lcw, c = e & (cw - 1);
      const int col = kx0 + c;
      if (col < hx) uo[(int64_t)y * tp + col] = buf[mul24(c, ld) + y];
    }
    __syncthreads();   // the next item refills buf, kr and tw
  }
}

// ---------------------------------------------------------------- kernel row DFTs
// kr[kx][fr][yy] = sum_x K_fr[yy][x] exp(-2 pi i kx x / Px) for every
// half-spectrum column kx < hx (zero for yy >= k_fr), in FP64 from the FP64
// twiddle table, rounded once to T: the column pass evaluates each kernel's
// spectrum at (ky, kx) from these along y.  Once per frame, shared by its
// channels.  Items: 256 consecutive entries of [0, hx * 2 * CBP_MAX_K).
static_assert(2 * CBP_MAX_K == 64, "one column's entries fill one wave");

template <typename T>
__global__ __launch_bounds__(256) void k_kernel_dft(batch_ref br) {
  for_items<Q_KRDFT>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int e = item * 256 + (int)threadIdx.x;
    const int hx = d.hx, Px = d.Px;
    if (e >= hx * 2 * CBP_MAX_K) return;
    // a wave's 64 entries share one column kx (2 CBP_MAX_K = 64): its
    // twiddles are wave-uniform (scalar loads)
    const int kx = __builtin_amdgcn_readfirstlane(e / (2 * CBP_MAX_K)), rem = e - kx * 2 * CBP_MAX_K;
    const int fr = rem / CBP_MAX_K, yy = rem - fr * CBP_MAX_K;
    const int k = fr ? d.k2 : d.k1;
    const double* K = fr ? d.K2 : d.K1;
    const c64* twd = d.twxd;
    double sr = 0.0, si = 0.0;
    if (yy < k) {
      // eight (twiddle, coefficient) pairs loaded per batch, summed in x order
      int t = 0;
      for (int x0 = 0; x0 < k; x0 += 8) {
        c64 w[8];
        double kv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          w[u] = twd[t];
          kv[u] = K[yy * k + min(x0 + u, k - 1)];
          t += kx;
          if (t >= Px) t -= Px;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (x0 + u < k) {
            sr += kv[u] * w[u].re;
            si += kv[u] * w[u].im;
          }
      }
    }
    ((cplx<T>*)d.kr)[e] = {T(sr), T(si)};
  });
}

// ---------------------------------------------------------------- pass 3
// Items: (pair of output rows, channel).  A workgroup that owns several items
// loads the next item's spectra into registers while it transforms the
// current one.
template <typename T>
__global__ __launch_bounds__(256) void k_row_inv(batch_ref br) {
  extern __shared__ __attribute__((aligned(16))) char sm_ri[];
  __shared__ int st[BATCH_CHUNK + 1];
  const int nf = br.nframes;
  const int* sq = br.starts + (size_t)Q_ROW_INV * (nf + 1);
  for (int t = threadIdx.x; t <= nf; t += blockDim.x) st[t] = sq[t];
  __syncthreads();
  int first, end, step;
  xcd_items(__builtin_amdgcn_readfirstlane(st[nf]), (int)blockIdx.x, (int)gridDim.x, first, end, step);
  auto frame_of = [&](int it) __attribute__((always_inline)) {
    int lo = 0, hi = nf;   // st[lo] <= it < st[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (st[mid] <= it) lo = mid;
      else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
  };
  auto desc = [&](int fi) __attribute__((always_inline)) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) frame_desc cdesc;
    return ((const cdesc*)br.descs)[fi];
#else
    return br.descs[fi];
#endif
  };
  // the spectra of item it's two rows into registers: entry k < hx read
  // directly, k >= hx as the conjugate of entry N - k (< hx); indices past N
  // clamp to 0 and are discarded
  cplx<T> Av[8], Bv[8];
  auto fetch = [&](int it) __attribute__((always_inline)) {
    const int fi = frame_of(it);
    const frame_desc d = desc(fi);
    const int item = it - __builtin_amdgcn_readfirstlane(st[fi]);
    const int N = d.fx.N, hx = d.hx, m = d.m;
    const int npair = (m + 1) / 2;
    const int ya = 2 * (item % npair), ch = item / npair;
    const cplx<T>* ua = (const cplx<T>*)d.u + (int64_t)ch * m * d.hxp + (int64_t)ya * d.hxp;
    const cplx<T>* ubv = ya + 1 < m ? ua + d.hxp : ua;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = t * 256 + (int)threadIdx.x;
      const int kk = k < hx ? k : max(N - k, 0);
      Av[t] = ua[kk];
      Bv[t] = ubv[kk];
    }
  };
  if (first < end) fetch(first);
  int tabN = 0;                  // plan of the pass tables in LDS (length,
  unsigned long long tabCode = 0;  // pass order)
  for (int it = first; it < end; it += step) {
    const int fi = frame_of(it);
    const frame_desc d = desc(fi);
    const int item = it - __builtin_amdgcn_readfirstlane(st[fi]);
    const fft_plan& px = d.fx;
    const int N = px.N, hx = d.hx, m = d.m, n = d.n;
    const T scale = (T)(1.0 / ((double)d.Py * (double)d.Px));
    cplx<T>* a = (cplx<T>*)sm_ri;
    cplx<T>* twf = a + N;
    pass_twiddles(twf, px, tabN, tabCode);
    const int npair = (m + 1) / 2;
    const int ya = 2 * (item % npair), yb = ya + 1, ch = item / npair;
    const bool hb = yb < m;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = t * 256 + (int)threadIdx.x;
      if (k < N) {
        cplx<T> A = Av[t], B = hb ? Bv[t] : cplx<T>{T(0), T(0)};
        if (k >= hx) { A = conj(A); B = conj(B); }
        if ((k == 0) || (2 * k == N)) { A.im = T(0); B.im = T(0); }
        a[k] = {A.re - B.im, A.im + B.re};   // A + i B
      }
    }
    __syncthreads();
    // the next item's spectra are in flight while this one is transformed
    if (it + step < end) fetch(it + step);
    ip_fft<+1, 256, ROW_MAXE, true>(a, N, px, twf, 1);
    const cplx<T>* z = a;
    T* oa = (T*)d.out + ch * d.ocs + (int64_t)ya * d.opitch;
    T* ob = oa + d.opitch;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
      oa[x] = z[x].re * scale;
      if (hb) ob[x] = z[x].im * scale;
    }
    __syncthreads();
  }
}

}  // namespace

// a row and the plan's pass twiddle tables (twn entries)
size_t row_lds_bytes(int N, int twn, int esize) { return ((size_t)N + (size_t)twn) * 2 * esize; }
// the strip (column stride col_ld <= N + 15), the kernels' row DFTs, the
// full twiddle table and twn more entries (col_table_entries: the filter's
// w_N^(g y) and the plan's pass twiddle tables)
size_t col_lds_bytes(int N, int cw, int twn, int esize) {
  return ((size_t)cw * (N + 15) + (size_t)cw * 2 * CBP_MAX_K + (size_t)N + (size_t)twn) * 2 * esize;
}

// Threads of the column-pass workgroup for a strip of cw * N entries: the
// fewest of 256 / 512 / 1024 whose registers hold the strip with at least
// one wave per column (cw <= NT / 64).
int col_threads(int N, int cw, int esize) {
  const int64_t e = (int64_t)cw * N;
  const int l256 = esize == 4 ? col_max_elems<float, 256>() : col_max_elems<double, 256>();
  const int l512 = esize == 4 ? col_max_elems<float, 512>() : col_max_elems<double, 512>();
  if (cw <= 4 && e <= l256) return 256;
  return (cw <= 8 && e <= l512) ? 512 : 1024;
}

int col_max_strip_elems(int esize) { return esize == 4 ? col_max_elems<float, 1024>() : col_max_elems<double, 1024>(); }

// Resident row-pass workgroups per CU (its registers and lds bytes of LDS),
// for the persistent grid: a workgroup beyond that would start only when
// another ends and leave a tail.  Kept per (element size, LDS in 4 KiB steps).
int row_fwd_per_cu(size_t lds, int esize) {
  static std::atomic<int> cache[2][41];
  const int b = std::min((int)((lds + 4095) / 4096), 40);
  std::atomic<int>& c = cache[esize == 8][b];
  int n = c.load(std::memory_order_relaxed);
  if (n > 0) return n;
  const void* f = esize == 8 ? (const void*)k_row_fwd<double> : (const void*)k_row_fwd<float>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 256, (size_t)b * 4096) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return 1;
  }
  c.store(n, std::memory_order_relaxed);
  return n;
}

// Resident column-pass workgroups per CU for strips of cw columns of length
// N (its variant's registers and LDS), for the persistent grid.  Kept per
// (element size, variant, LDS in 4 KiB steps).
// The column-pass instance of element type T, workgroup size nt and filter
// group g.
template <typename T>
const void* col_kernel(int nt, int g) {
  if (nt == 256)
    return g == 4 ? (const void*)k_col_filter<T, 256, 4> : g == 2 ? (const void*)k_col_filter<T, 256, 2>
                                                                   : (const void*)k_col_filter<T, 256, 1>;
  if (nt == 512)
    return g == 4 ? (const void*)k_col_filter<T, 512, 4> : g == 2 ? (const void*)k_col_filter<T, 512, 2>
                                                                   : (const void*)k_col_filter<T, 512, 1>;
  return g == 4 ? (const void*)k_col_filter<T, 1024, 4> : g == 2 ? (const void*)k_col_filter<T, 1024, 2>
                                                                  : (const void*)k_col_filter<T, 1024, 1>;
}

int col_per_cu(int N, int cw, int twn, int g, int esize) {
  static std::atomic<int> cache[2][3][3][41];
  const int nt = col_threads(N, cw, esize);
  const int v = nt == 256 ? 0 : nt == 512 ? 1 : 2;
  const int gi = g == 4 ? 0 : g == 2 ? 1 : 2;
  const int b = std::min((int)((col_lds_bytes(N, cw, twn, esize) + 4095) / 4096), 40);
  std::atomic<int>& c = cache[esize == 8][v][gi][b];
  int n = c.load(std::memory_order_relaxed);
  if (n > 0) return n;
  const void* f = esize == 8 ? col_kernel<double>(nt, g) : col_kernel<float>(nt, g);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, nt, (size_t)b * 4096) != hipSuccess ||
      n < 1) {
    (void)hipGetLastError();
    return 1;
  }
  c.store(n, std::memory_order_relaxed);
  return n;
}

void set_fft_attrs() {
  const void* fns[4] = {(const void*)k_row_fwd<float>, (const void*)k_row_inv<float>, (const void*)k_row_fwd<double>,
                        (const void*)k_row_inv<double>};
  for (const void* f : fns) hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  for (int nt : {256, 512, 1024})
    for (int g : {4, 2, 1}) {
      hipFuncSetAttribute(col_kernel<float>(nt, g), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      hipFuncSetAttribute(col_kernel<double>(nt, g), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }
}

template <typename T>
hipError_t launch_row_fwd(const batch_ref& br, int grid, int maxPx, int maxTw, int with_ey, hipStream_t st) {
  prof_begin(PH_ROW_FWD, st);
  hipLaunchKernelGGL(k_row_fwd<T>, dim3(grid), dim3(256), row_lds_bytes(maxPx, maxTw, (int)sizeof(T)), st, br,
                     with_ey);
  prof_end(PH_ROW_FWD, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col(const batch_ref& br, int grid, int maxPy, int maxcw, int maxTw, int gmask, hipStream_t st) {
  prof_begin(PH_COL_FILTER, st);
  const size_t lds = col_lds_bytes(maxPy, maxcw, maxTw, (int)sizeof(T));
  const int nt = col_threads(maxPy, maxcw, (int)sizeof(T));
  void* args[] = {(void*)&br};
  hipError_t e = hipSuccess;
  for (int g : {4, 2, 1})
    if ((gmask >> g & 1) && e == hipSuccess) e = hipLaunchKernel(col_kernel<T>(nt, g), dim3(grid), dim3(nt), args, lds, st);
  prof_end(PH_COL_FILTER, st);
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
hipError_t launch_kernel_dft(const batch_ref& br, int grid, hipStream_t st) {
  prof_begin(PH_KR_DFT, st);
  hipLaunchKernelGGL(k_kernel_dft<T>, dim3(grid), dim3(256), 0, st, br);
  prof_end(PH_KR_DFT, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row_inv(const batch_ref& br, int grid, int maxPx, int maxTw, hipStream_t st) {
  prof_begin(PH_ROW_INV, st);
  hipLaunchKernelGGL(k_row_inv<T>, dim3(grid), dim3(256), row_lds_bytes(maxPx, maxTw, (int)sizeof(T)), st, br);
  prof_end(PH_ROW_INV, st);
  return hipGetLastError();
}


template hipError_t launch_row_fwd<float>(const batch_ref&, int, int, int, int, hipStream_t);
template hipError_t launch_row_fwd<double>(const batch_ref&, int, int, int, int, hipStream_t);
template hipError_t launch_col<float>(const batch_ref&, int, int, int, int, int, hipStream_t);
template hipError_t launch_col<double>(const batch_ref&, int, int, int, int, int, hipStream_t);
template hipError_t launch_kernel_dft<float>(const batch_ref&, int, hipStream_t);
template hipError_t launch_kernel_dft<double>(const batch_ref&, int, hipStream_t);
template hipError_t launch_row_inv<float>(const batch_ref&, int, int, int, hipStream_t);
template hipError_t launch_row_inv<double>(const batch_ref&, int, int, int, hipStream_t);

}  // namespace cbp
