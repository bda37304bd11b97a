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
//   3. inverse row pass: two rows of U packed as one complex spectrum (each
//      completed by Hermitian symmetry), one inverse FFT, real / imaginary
//      parts are the two output rows, scaled by 1/(Py Px), cropped to n.
// T is float (mixed form) or double (FP64 form).
#include "eigsmall.h"
#include "internal.h"

namespace cbp {

namespace {

// The split twiddle tables of an N-point transform (fft_core.h tw_split) into
// LDS: lo[i] = w_N^i, i < 64, and hi[j] = w_N^{64 j}, j < ceil(N / 64), each an
// FP64 sincospi rounded once to T.  The passes read them from LDS instead of
// a table in global memory.
template <typename T>
__device__ inline tw_split<T> split_twiddles(cplx<T>* lo, cplx<T>* hi, int N) {
  const int nhi = (N + 63) >> 6;
  for (int t = threadIdx.x; t < 64 + nhi; t += blockDim.x) {
    const int e = t < 64 ? t : 64 * (t - 64);
    double sn, cs;
    sincospi(-2.0 * (double)e / (double)N, &sn, &cs);
    (t < 64 ? lo[t] : hi[t - 64]) = {T(cs), T(sn)};
  }
  return tw_split<T>{lo, hi};
}

// Run all passes of plan p on nbatch transforms (stride bstride) held in a;
// b is the ping-pong partner.  Returns the buffer holding the result.
template <int DIR, typename T, typename Tab>
__device__ __attribute__((always_inline)) inline cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, const fft_plan& p, const Tab& tw, int nbatch,
                                   int bstride) {
  cplx<T>* src = a;
  cplx<T>* dst = b;
  int Ns = 1;
  for (int s = 0; s < p.npass; ++s) {
    const int R = plan_radix(p, s);
    fft_pass<DIR>(src, dst, p.N, R, Ns, tw, nbatch, bstride, threadIdx.x, blockDim.x);
    __syncthreads();
    cplx<T>* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  return src;
}

// ---------------------------------------------------------------- pass 1
// Items: (row y, channel).  With with_ey, the unit-circle evaluation of both
// rows (fold modulo S and S-point DFT, as k_eval_rows: the same lanes, the
// same order, hence the same bits) is taken from the row in LDS; waves 0-3
// fold (frame, residue parity) = (w & 1, w >> 1).
template <typename T>
// Workgroups [0, gr) run the row pass; the rest run the column evaluation
// (its scratch carved from the dynamic LDS).
__global__ __launch_bounds__(256) void k_row_fwd(batch_ref br, int with_ey, int gr) {
  extern __shared__ __attribute__((aligned(16))) char sm_rf[];
  __shared__ cplx<T> twl[64], twh[CBP_MAX_FFT_F32 / 64];
  __shared__ double gy[2][CBP_MAX_S];
  __shared__ double fpart_l[2][64];
  __shared__ c64 twS[CBP_MAX_S];
  if ((int)blockIdx.x >= gr) {
    double(*F)[16] = (double(*)[16])sm_rf;
    c64* twe = (c64*)(sm_rf + (size_t)CBP_MAX_S * 16 * sizeof(double));
    for_items_part<Q_EVAL_COLS>(br, (int)blockIdx.x - gr, (int)gridDim.x - gr,
                                [&](const frame_desc& d, int item) __attribute__((always_inline)) {
                                  eval_cols_item(d, item, F, twe);
                                });
    return;
  }
  for_items_part<Q_ROW_FWD>(br, (int)blockIdx.x, gr, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const fft_plan& px = d.fx;
    const int N = px.N, hx = d.hx;
    cplx<T>* a = (cplx<T>*)sm_rf;
    cplx<T>* b = a + N;
    const tw_split<T> tw = split_twiddles(twl, twh, N);
    const int y = item % d.Hmax, ch = item / d.Hmax;
    // row pointers clamped to each frame's last row (rows past it read as zero)
    const T* r1 = (const T*)d.b1 + ch * d.cs1 + (int64_t)min(y, d.H1 - 1) * d.p1;
    const T* r2 = (const T*)d.b2 + ch * d.cs2 + (int64_t)min(y, d.H2 - 1) * d.p2;
    const bool in1 = y < d.H1, in2 = y < d.H2;
    if (with_ey)
      for (int t = threadIdx.x; t < d.S; t += blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * (double)t / (double)d.S, &sn, &cs);
        twS[t] = {cs, sn};
      }
    // eight loads per frame and thread in flight, from clamped (always valid)
    // addresses; entries outside the frame are zeroed afterwards
    {
      const int W1 = d.W1, W2 = d.W2;
      for (int x0 = 0; x0 < N; x0 += 8 * (int)blockDim.x) {
        T uv[8], wv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int x = x0 + t * (int)blockDim.x + (int)threadIdx.x;
          uv[t] = r1[min(x, W1 - 1)];
          wv[t] = r2[min(x, W2 - 1)];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int x = x0 + t * (int)blockDim.x + (int)threadIdx.x;
          if (x < N) a[x] = {(in1 && x < W1) ? uv[t] : T(0), (in2 && x < W2) ? wv[t] : T(0)};
        }
      }
    }
    __syncthreads();
    if (with_ey) {
      // the row evaluation of both rows (k_eval_rows's lanes and order):
      // wave fr folds frame fr's row into partials, lane g S + r summing
      // x = r + S (g + G i); the residues then add their G partials in order
      const int S = d.S, G = 64 / S;
      const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
      const int gl = l / S, r = l - gl * S;
      if (wv < 2) {
        const int W = wv ? d.W2 : d.W1;
        double acc = 0.0;
        if ((wv ? in2 : in1) && gl < G)
          for (int x = r + S * gl; x < W; x += S * G) acc += (double)(wv ? a[x].im : a[x].re);
        fpart_l[wv][l] = acc;
      }
      __syncthreads();
      if (wv < 2 && l < S) {
        double sr = fpart_l[wv][l];
        for (int q = 1; q < G; ++q) sr += fpart_l[wv][q * S + l];
        gy[wv][l] = sr;
      }
      __syncthreads();
      if (wv < 2 && l < S && (wv ? in2 : in1)) {
        const int fr = wv;
        c64 e = {0.0, 0.0};
        int t = 0;
        for (int rr = 0; rr < S; ++rr) {
          const double f = gy[fr][rr];
          e.re += f * twS[t].re;
          e.im += f * twS[t].im;
          t += l;
          if (t >= S) t -= S;
        }
        d.ey[((size_t)(2 * ch + fr) * S + l) * d.Hmax + y] = e;
      }
    }
    const cplx<T>* z = fft_lds<-1>(a, b, px, tw, 1, N);
    cplx<T>* o1 = (cplx<T>*)d.t1 + (int64_t)ch * d.Hmax * hx + (int64_t)y * hx;
    cplx<T>* o2 = (cplx<T>*)d.t2 + (int64_t)ch * d.Hmax * hx + (int64_t)y * hx;
    for (int k = threadIdx.x; k < hx; k += blockDim.x) {
      const cplx<T> zk = z[k];
      const cplx<T> zn = conj(z[k == 0 ? 0 : N - k]);
      const cplx<T> s = zk + zn, df = zk - zn;
      if (in1) o1[k] = {T(0.5) * s.re, T(0.5) * s.im};       // (Z_k + conj Z_{N-k}) / 2
      if (in2) o2[k] = {T(0.5) * df.im, T(-0.5) * df.re};    // (Z_k - conj Z_{N-k}) / (2i)
    }
  });
}

// ---------------------------------------------------------------- pass 2
// Items: (strip of cw columns, channel).
template <typename T>
__global__ __launch_bounds__(256) void k_col_filter(batch_ref br) {
  extern __shared__ __attribute__((aligned(16))) char sm_cf[];
  __shared__ cplx<T> twl[64], twh[CBP_MAX_FFT_F32 / 64];
  for_items<Q_COL>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const fft_plan& py = d.fy;
    const int N = py.N, cw = d.cw, hx = d.hx, m = d.m;
    const int k1 = d.k1, k2 = d.k2, Px = d.Px, H1 = d.H1, H2 = d.H2;
    const double* K1 = d.K1;
    const double* K2 = d.K2;
    const c64* twd = d.twxd;
    const T lam = (T)d.lambda;
    const bool two = !(d.variant & VAR_DIVIDE_B1);   // two-channel division, or B1 / K1 alone
    const int nf = 2 * cw;                      // transforms in flight: (column, frame)
    cplx<T>* a = (cplx<T>*)sm_cf;               // [nf][N]
    cplx<T>* b = a + (size_t)nf * N;            // [nf][N]
    const tw_split<T> tw = split_twiddles(twl, twh, N);
    cplx<T>* kr = b + (size_t)nf * N;           // [cw][2][CBP_MAX_K] row DFTs of the kernels at kx
    const int nstrip = (hx + cw - 1) / cw;
    const int kx0 = (item % nstrip) * cw, ch = item / nstrip;
    const int64_t tpc = (int64_t)d.Hmax * hx;
    const cplx<T>* s1 = (const cplx<T>*)d.t1 + ch * tpc;
    const cplx<T>* s2 = (const cplx<T>*)d.t2 + ch * tpc;
    // load: element (y, f) with f = 2*col + frame; consecutive threads walk f
    // (adjacent columns of one row) for coalescing
    const int lnf = __builtin_ctz(nf);         // cw, hence nf, is a power of two
    // eight loads per thread in flight from clamped (always valid) addresses;
    // entries outside the frame or past the last column are zeroed afterwards
    for (int e0 = 0; e0 < nf * N; e0 += 8 * (int)blockDim.x) {
      cplx<T> v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int e = e0 + t * (int)blockDim.x + (int)threadIdx.x;
        const int y = e >> lnf, f = e & (nf - 1);
        const int col = min(kx0 + (f >> 1), hx - 1);
        const int fr = f & 1;
        const cplx<T>* src = fr ? s2 : s1;
        v[t] = src[(int64_t)min(y, (fr ? H2 : H1) - 1) * hx + col];
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int e = e0 + t * (int)blockDim.x + (int)threadIdx.x;
        const int y = e >> lnf, f = e & (nf - 1);
        const int fr = f & 1;
        if (e < nf * N) {
          const bool in = kx0 + (f >> 1) < hx && y < (fr ? H2 : H1);
          a[(size_t)f * N + y] = in ? v[t] : cplx<T>{T(0), T(0)};
        }
      }
    }
    // kernel row DFTs at this strip's columns: kr[c][fr][yy] = sum_x K[yy][x] exp(-2 pi i kx x / Px)
    for (int e = threadIdx.x; e < cw * 2 * CBP_MAX_K; e += blockDim.x) {
      const int c = e / (2 * CBP_MAX_K), rem = e - c * 2 * CBP_MAX_K;
      const int fr = rem / CBP_MAX_K, yy = rem - fr * CBP_MAX_K;
      const int k = fr ? k2 : k1;
      const double* K = fr ? K2 : K1;
      const int kx = kx0 + c;
      double sr = 0.0, si = 0.0;
      if (yy < k && kx < hx) {
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
      kr[e] = {T(sr), T(si)};
    }
    __syncthreads();
    cplx<T>* f1 = fft_lds<-1>(a, b, py, tw, nf, N);
    cplx<T>* f2 = (f1 == a) ? b : a;
    // filter: combined spectrum written into the frame-1 slot of each column
    const float rN = 1.0f / (float)N;
    const int kmax = k1 > k2 ? k1 : k2;
    for (int e = threadIdx.x; e < cw * N; e += blockDim.x) {
      const int c = fdiv_floor(e, rN), ky = e - c * N;
      // kernel spectra at (ky, kx): sum_yy kr[yy] z^yy, z = exp(-2 pi i ky / Py),
      // by Horner's rule (kr is zero beyond each kernel's size)
      const cplx<T>* kr1 = kr + (size_t)c * 2 * CBP_MAX_K;
      const cplx<T>* kr2 = kr1 + CBP_MAX_K;
      const cplx<T> z = tw[ky];
      cplx<T> kh1 = kr1[kmax - 1], kh2 = kr2[kmax - 1];
      for (int yy = kmax - 2; yy >= 0; --yy) {
        kh1 = kh1 * z + kr1[yy];
        kh2 = kh2 * z + kr2[yy];
      }
      const cplx<T> B1 = f1[(size_t)(2 * c) * N + ky];
      const cplx<T> B2 = f1[(size_t)(2 * c + 1) * N + ky];
      const cplx<T> num = two ? cmulc(kh1, B1) + cmulc(kh2, B2) : cmulc(kh1, B1);
      const T kk = two ? norm2(kh1) + norm2(kh2) : norm2(kh1);
      const T den = kk + lam;
      const T inv = den > T(0) ? T(1) / den : T(0);
      // where both kernel spectra vanish (a zeroed kernel pair) the
      // quotient is zero, whatever the frames hold
      f1[(size_t)(2 * c) * N + ky] = kk > T(0) ? cplx<T>{num.re * inv, num.im * inv} : cplx<T>{T(0), T(0)};
    }
    __syncthreads();
    // inverse column FFT of the cw combined spectra (slots 0, 2, 4, ...)
    const cplx<T>* r = fft_lds<+1>(f1, f2, py, tw, cw, 2 * N);
    cplx<T>* uo = (cplx<T>*)d.u + (int64_t)ch * m * hx;
    const int lcw = __builtin_ctz(cw);
    for (int e = threadIdx.x; e < m * cw; e += blockDim.x) {
      const int y = e >> lcw, c = e & (cw - 1);
      const int col = kx0 + c;
      if (col < hx) uo[(int64_t)y * hx + col] = r[(size_t)(2 * c) * N + y];
    }
  });
}

// ---------------------------------------------------------------- pass 3
// Items: (pair of output rows, channel).
template <typename T>
__global__ __launch_bounds__(256) void k_row_inv(batch_ref br) {
  extern __shared__ __attribute__((aligned(16))) char sm_ri[];
  __shared__ cplx<T> twl[64], twh[CBP_MAX_FFT_F32 / 64];
  for_items<Q_ROW_INV>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const fft_plan& px = d.fx;
    const int N = px.N, hx = d.hx, m = d.m, n = d.n;
    const T scale = (T)(1.0 / ((double)d.Py * (double)d.Px));
    cplx<T>* a = (cplx<T>*)sm_ri;
    cplx<T>* b = a + N;
    const tw_split<T> tw = split_twiddles(twl, twh, N);
    const int npair = (m + 1) / 2;
    const int ya = 2 * (item % npair), yb = ya + 1, ch = item / npair;
    const cplx<T>* ua = (const cplx<T>*)d.u + (int64_t)ch * m * hx + (int64_t)ya * hx;
    const cplx<T>* ub = ua + hx;
    const bool hb = yb < m;
    // eight index pairs per thread in flight: entry k < hx read directly,
    // k >= hx as the conjugate of entry N - k (< hx); indices past N clamp
    // to 0 and are discarded
    const cplx<T>* ubv = hb ? ub : ua;
    for (int k0 = 0; k0 < N; k0 += 8 * (int)blockDim.x) {
      cplx<T> Av[8], Bv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = k0 + t * (int)blockDim.x + (int)threadIdx.x;
        const int kk = k < hx ? k : max(N - k, 0);
        Av[t] = ua[kk];
        Bv[t] = ubv[kk];
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = k0 + t * (int)blockDim.x + (int)threadIdx.x;
        if (k < N) {
          cplx<T> A = Av[t], B = hb ? Bv[t] : cplx<T>{T(0), T(0)};
          if (k >= hx) { A = conj(A); B = conj(B); }
          if ((k == 0) || (2 * k == N)) { A.im = T(0); B.im = T(0); }
          a[k] = {A.re - B.im, A.im + B.re};   // A + i B
        }
      }
    }
    __syncthreads();
    const cplx<T>* z = fft_lds<+1>(a, b, px, tw, 1, N);
    T* oa = (T*)d.out + ch * d.ocs + (int64_t)ya * d.opitch;
    T* ob = oa + d.opitch;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
      oa[x] = z[x].re * scale;
      if (hb) ob[x] = z[x].im * scale;
    }
  });
}

}  // namespace

size_t row_lds_bytes(int N, int esize) { return (size_t)2 * N * 2 * esize; }
size_t col_lds_bytes(int N, int cw, int esize) {
  return ((size_t)(4 * cw) * N + (size_t)cw * 2 * CBP_MAX_K) * 2 * esize;
}

void set_fft_attrs() {
  const void* fns[6] = {(const void*)k_row_fwd<float>, (const void*)k_col_filter<float>, (const void*)k_row_inv<float>,
                        (const void*)k_row_fwd<double>, (const void*)k_col_filter<double>,
                        (const void*)k_row_inv<double>};
  for (const void* f : fns) hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <typename T>
hipError_t launch_row_fwd(const batch_ref& br, int grid, int maxPx, int with_ey, int eval_grid,
                          hipStream_t st) {
  prof_begin(PH_ROW_FWD, st);
  size_t lds = row_lds_bytes(maxPx, (int)sizeof(T));
  if (eval_grid > 0 && lds < kEvalColsLds) lds = kEvalColsLds;
  hipLaunchKernelGGL(k_row_fwd<T>, dim3(grid + eval_grid), dim3(256), lds, st, br, with_ey, grid);
  prof_end(PH_ROW_FWD, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col(const batch_ref& br, int grid, int maxPy, int maxcw, hipStream_t st) {
  prof_begin(PH_COL_FILTER, st);
  hipLaunchKernelGGL(k_col_filter<T>, dim3(grid), dim3(256), col_lds_bytes(maxPy, maxcw, (int)sizeof(T)), st, br);
  prof_end(PH_COL_FILTER, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row_inv(const batch_ref& br, int grid, int maxPx, hipStream_t st) {
  prof_begin(PH_ROW_INV, st);
  hipLaunchKernelGGL(k_row_inv<T>, dim3(grid), dim3(256), row_lds_bytes(maxPx, (int)sizeof(T)), st, br);
  prof_end(PH_ROW_INV, st);
  return hipGetLastError();
}


template hipError_t launch_row_fwd<float>(const batch_ref&, int, int, int, int, hipStream_t);
template hipError_t launch_row_fwd<double>(const batch_ref&, int, int, int, int, hipStream_t);
template hipError_t launch_col<float>(const batch_ref&, int, int, int, hipStream_t);
template hipError_t launch_col<double>(const batch_ref&, int, int, int, hipStream_t);
template hipError_t launch_row_inv<float>(const batch_ref&, int, int, hipStream_t);
template hipError_t launch_row_inv<double>(const batch_ref&, int, int, hipStream_t);

}  // namespace cbp
