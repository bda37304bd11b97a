// Two-channel regularised Fourier division (Sec. 4: the latent is obtained by
// dividing a blurred frame by the recovered kernel in the Fourier domain;
// Sec. 5: an inverse FFT of the divided spectrum).  Over a Py x Px grid that
// covers both frames (no wrap-around of the full convolutions):
//   Lhat = (conj(K1hat) B1hat + conj(K2hat) B2hat) / (|K1hat|^2 + |K2hat|^2 + lambda),
//   L    = IFFT2(Lhat) cropped to m x n.
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
#include "internal.h"

namespace cbp {

namespace {

template <typename T>
__device__ inline void fft_twiddles(cplx<T>* tw, int N) {
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)N, &s, &c);
    tw[t] = {T(c), T(s)};
  }
}

// Run all passes of plan p on nbatch transforms (stride bstride) held in a;
// b is the ping-pong partner.  Returns the buffer holding the result.
template <int DIR, typename T>
__device__ inline cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, const fft_plan& p, const cplx<T>* tw, int nbatch,
                                   int bstride) {
  cplx<T>* src = a;
  cplx<T>* dst = b;
  int Ns = 1;
  for (int s = 0; s < p.npass; ++s) {
    const int R = p.radix[s];
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
template <typename T>
__global__ __launch_bounds__(256) void k_row_fwd(pair_view<T> v, fft_plan px, int hx, cplx<T>* t1, cplx<T>* t2,
                                                 int64_t tpitch_ch) {
  extern __shared__ __attribute__((aligned(16))) char sm_rf[];
  const int N = px.N;
  cplx<T>* a = (cplx<T>*)sm_rf;
  cplx<T>* b = a + N;
  cplx<T>* tw = b + N;
  const int y = blockIdx.x, ch = blockIdx.y;
  const T* r1 = v.b1 + ch * v.cs1 + (int64_t)y * v.p1;
  const T* r2 = v.b2 + ch * v.cs2 + (int64_t)y * v.p2;
  const bool in1 = y < v.H1, in2 = y < v.H2;
  fft_twiddles(tw, N);
  for (int x = threadIdx.x; x < N; x += blockDim.x) {
    const T u = (in1 && x < v.W1) ? r1[x] : T(0);
    const T w = (in2 && x < v.W2) ? r2[x] : T(0);
    a[x] = {u, w};
  }
  __syncthreads();
  const cplx<T>* z = fft_lds<-1>(a, b, px, tw, 1, N);
  cplx<T>* o1 = t1 + ch * tpitch_ch + (int64_t)y * hx;
  cplx<T>* o2 = t2 + ch * tpitch_ch + (int64_t)y * hx;
  for (int k = threadIdx.x; k < hx; k += blockDim.x) {
    const cplx<T> zk = z[k];
    const cplx<T> zn = conj(z[k == 0 ? 0 : N - k]);
    const cplx<T> s = zk + zn, d = zk - zn;
    if (in1) o1[k] = {T(0.5) * s.re, T(0.5) * s.im};     // (Z_k + conj Z_{N-k}) / 2
    if (in2) o2[k] = {T(0.5) * d.im, T(-0.5) * d.re};    // (Z_k - conj Z_{N-k}) / (2i)
  }
}

// ---------------------------------------------------------------- pass 2
template <typename T>
__global__ __launch_bounds__(256) void k_col_filter(const cplx<T>* t1, const cplx<T>* t2, int H1, int H2, int hx,
                                                    int64_t tpitch_ch, cplx<T>* u, int m, int64_t upitch_ch,
                                                    const double* K1, int k1, const double* K2, int k2, int Px,
                                                    fft_plan py, T lam, int cw) {
  extern __shared__ __attribute__((aligned(16))) char sm_cf[];
  const int N = py.N;
  const int nf = 2 * cw;                      // transforms in flight: (column, frame)
  cplx<T>* a = (cplx<T>*)sm_cf;               // [nf][N]
  cplx<T>* b = a + (size_t)nf * N;            // [nf][N]
  cplx<T>* tw = b + (size_t)nf * N;           // [N]
  cplx<T>* kr = tw + N;                       // [cw][2][CBP_MAX_K] row DFTs of the kernels at kx
  const int kx0 = blockIdx.x * cw, ch = blockIdx.y;
  const cplx<T>* s1 = t1 + ch * tpitch_ch;
  const cplx<T>* s2 = t2 + ch * tpitch_ch;
  fft_twiddles(tw, N);
  // load: element (y, f) with f = 2*col + frame; consecutive threads walk f
  // (adjacent columns of one row) for coalescing
  for (int e = threadIdx.x; e < nf * N; e += blockDim.x) {
    const int y = e / nf, f = e - y * nf;
    const int col = kx0 + (f >> 1);
    const int fr = f & 1;
    cplx<T> val = {T(0), T(0)};
    if (col < hx) {
      if (fr == 0 && y < H1) val = s1[(int64_t)y * hx + col];
      if (fr == 1 && y < H2) val = s2[(int64_t)y * hx + col];
    }
    a[(size_t)f * N + y] = val;
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
      int64_t t = 0;
      for (int x = 0; x < k; ++x) {
        double sn, cs;
        sincospi(-2.0 * (double)t / (double)Px, &sn, &cs);
        const double kv = K[yy * k + x];
        sr += kv * cs;
        si += kv * sn;
        t += kx;
        if (t >= Px) t -= Px;
      }
    }
    kr[e] = {T(sr), T(si)};
  }
  __syncthreads();
  cplx<T>* f1 = fft_lds<-1>(a, b, py, tw, nf, N);
  cplx<T>* f2 = (f1 == a) ? b : a;
  // filter: combined spectrum written into the frame-1 slot of each column
  for (int e = threadIdx.x; e < cw * N; e += blockDim.x) {
    const int c = e / N, ky = e - c * N;
    cplx<T> kh1 = {T(0), T(0)}, kh2 = {T(0), T(0)};
    int t = 0;
    const cplx<T>* kr1 = kr + (size_t)c * 2 * CBP_MAX_K;
    const cplx<T>* kr2 = kr1 + CBP_MAX_K;
    const int kmax = k1 > k2 ? k1 : k2;
    for (int yy = 0; yy < kmax; ++yy) {
      const cplx<T> w = tw[t];
      if (yy < k1) kh1 = kh1 + kr1[yy] * w;
      if (yy < k2) kh2 = kh2 + kr2[yy] * w;
      t += ky;
      if (t >= N) t -= N;
    }
    const cplx<T> B1 = f1[(size_t)(2 * c) * N + ky];
    const cplx<T> B2 = f1[(size_t)(2 * c + 1) * N + ky];
    const cplx<T> num = cmulc(kh1, B1) + cmulc(kh2, B2);
    const T den = norm2(kh1) + norm2(kh2) + lam;
    const T inv = den > T(0) ? T(1) / den : T(0);
    f1[(size_t)(2 * c) * N + ky] = {num.re * inv, num.im * inv};
  }
  __syncthreads();
  // inverse column FFT of the cw combined spectra (slots 0, 2, 4, ...)
  const cplx<T>* r = fft_lds<+1>(f1, f2, py, tw, cw, 2 * N);
  cplx<T>* uo = u + ch * upitch_ch;
  for (int e = threadIdx.x; e < m * cw; e += blockDim.x) {
    const int y = e / cw, c = e - y * cw;
    const int col = kx0 + c;
    if (col < hx) uo[(int64_t)y * hx + col] = r[(size_t)(2 * c) * N + y];
  }
}

// ---------------------------------------------------------------- pass 3
template <typename T>
__global__ __launch_bounds__(256) void k_row_inv(const cplx<T>* u, int hx, int m, int64_t upitch_ch, fft_plan px,
                                                 T* out, int64_t opitch, int64_t ocs, int n, T scale) {
  extern __shared__ __attribute__((aligned(16))) char sm_ri[];
  const int N = px.N;
  cplx<T>* a = (cplx<T>*)sm_ri;
  cplx<T>* b = a + N;
  cplx<T>* tw = b + N;
  const int ya = 2 * blockIdx.x, yb = ya + 1, ch = blockIdx.y;
  const cplx<T>* ua = u + ch * upitch_ch + (int64_t)ya * hx;
  const cplx<T>* ub = u + ch * upitch_ch + (int64_t)yb * hx;
  const bool hb = yb < m;
  fft_twiddles(tw, N);
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    cplx<T> A, B;
    const bool edge = (k == 0) || (2 * k == N);
    if (k < hx) {
      A = ua[k];
      B = hb ? ub[k] : cplx<T>{T(0), T(0)};
    } else {
      A = conj(ua[N - k]);
      B = hb ? conj(ub[N - k]) : cplx<T>{T(0), T(0)};
    }
    if (edge) { A.im = T(0); B.im = T(0); }
    a[k] = {A.re - B.im, A.im + B.re};   // A + i B
  }
  __syncthreads();
  const cplx<T>* z = fft_lds<+1>(a, b, px, tw, 1, N);
  T* oa = out + ch * ocs + (int64_t)ya * opitch;
  T* ob = out + ch * ocs + (int64_t)yb * opitch;
  for (int x = threadIdx.x; x < n; x += blockDim.x) {
    oa[x] = z[x].re * scale;
    if (hb) ob[x] = z[x].im * scale;
  }
}

}  // namespace

size_t row_lds_bytes(int N, int esize) { return (size_t)3 * N * 2 * esize; }
size_t col_lds_bytes(int N, int cw, int esize) {
  return ((size_t)(4 * cw + 1) * N + (size_t)cw * 2 * CBP_MAX_K) * 2 * esize;
}

namespace {
void set_fft_attrs_once() {
  static bool done = false;
  if (done) return;
  const void* fns[6] = {(const void*)k_row_fwd<float>, (const void*)k_col_filter<float>, (const void*)k_row_inv<float>,
                        (const void*)k_row_fwd<double>, (const void*)k_col_filter<double>,
                        (const void*)k_row_inv<double>};
  for (const void* f : fns) hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  done = true;
}
}  // namespace

template <typename T>
hipError_t launch_row_fwd(const pair_view<T>& v, const frame_plan& fp, char* ws, hipStream_t st) {
  set_fft_attrs_once();
  cplx<T>* t1 = (cplx<T>*)(ws + fp.off_t1);
  cplx<T>* t2 = (cplx<T>*)(ws + fp.off_t2);
  const int64_t tpc = (int64_t)fp.Hmax * fp.hx;
  prof_begin(PH_ROW_FWD, st);
  hipLaunchKernelGGL(k_row_fwd<T>, dim3(fp.Hmax, v.nch), dim3(256), row_lds_bytes(fp.Px, (int)sizeof(T)), st, v,
                     fp.fx, fp.hx, t1, t2, tpc);
  prof_end(PH_ROW_FWD, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_inv(const pair_view<T>& v, const frame_plan& fp, char* ws, const double* K1, const double* K2,
                          T* out, int64_t opitch, int64_t ocs, double lambda, hipStream_t st) {
  set_fft_attrs_once();
  cplx<T>* t1 = (cplx<T>*)(ws + fp.off_t1);
  cplx<T>* t2 = (cplx<T>*)(ws + fp.off_t2);
  cplx<T>* u = (cplx<T>*)(ws + fp.off_u);
  const int64_t tpc = (int64_t)fp.Hmax * fp.hx;
  const int64_t upc = (int64_t)fp.m * fp.hx;
  const int es = (int)sizeof(T);
  prof_begin(PH_COL_FILTER, st);
  hipLaunchKernelGGL(k_col_filter<T>, dim3((fp.hx + fp.cw - 1) / fp.cw, v.nch), dim3(256),
                     col_lds_bytes(fp.Py, fp.cw, es), st, t1, t2, fp.H1, fp.H2, fp.hx, tpc, u, fp.m, upc, K1, fp.k1,
                     K2, fp.k2, fp.Px, fp.fy, (T)lambda, fp.cw);
  prof_end(PH_COL_FILTER, st);
  const T scale = (T)(1.0 / ((double)fp.Py * (double)fp.Px));
  prof_begin(PH_ROW_INV, st);
  hipLaunchKernelGGL(k_row_inv<T>, dim3((fp.m + 1) / 2, v.nch), dim3(256), row_lds_bytes(fp.Px, es), st, u, fp.hx,
                     fp.m, upc, fp.fx, out, opitch, ocs, fp.n, scale);
  prof_end(PH_ROW_INV, st);
  return hipGetLastError();
}

template hipError_t launch_row_fwd<float>(const pair_view<float>&, const frame_plan&, char*, hipStream_t);
template hipError_t launch_row_fwd<double>(const pair_view<double>&, const frame_plan&, char*, hipStream_t);
template hipError_t launch_col_inv<float>(const pair_view<float>&, const frame_plan&, char*, const double*,
                                          const double*, float*, int64_t, int64_t, double, hipStream_t);
template hipError_t launch_col_inv<double>(const pair_view<double>&, const frame_plan&, char*, const double*,
                                           const double*, double*, int64_t, int64_t, double, hipStream_t);

}  // namespace cbp
