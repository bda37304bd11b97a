// Mixed-radix (2, 3, 4, 5, 7, 8) Stockham autosort FFT passes.
//
// A length-N transform (N a product of the radices) runs as one pass per
// radix factor R.  Pass s with stride Ns (the product of the radices already
// applied) performs N/R butterflies; butterfly j reads the R inputs
// src[j + r*N/R], multiplies input r by the twiddle w_N^{r*k*N/(Ns*R)}
// (k = j mod Ns), applies an R-point DFT and writes its R outputs to
// dst[(j - k)*R + k + r*Ns].  After the last pass the result is in natural
// order (Stockham's autosort formulation; see Van Loan, "Computational
// Frameworks for the Fast Fourier Transform", SIAM 1992).
//
// DIR = -1 computes X[m] = sum_t x[t] exp(-2 pi i m t / N) (forward),
// DIR = +1 the same with +i (unnormalised inverse).  Twiddles tw[t] =
// exp(-2 pi i t / N), t in [0, N), come from a table (any type with
// operator[]).
//
// Everything here is host+device so the same butterfly code can be checked
// on the CPU.
#pragma once

#include "common.h"

namespace cbp {

// ---------------------------------------------------------------- R-point DFTs
template <int DIR, typename T>
CBP_HD void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <int DIR, typename T>
CBP_HD void dft4(cplx<T>& v0, cplx<T>& v1, cplx<T>& v2, cplx<T>& v3) {
  cplx<T> a = v0 + v2, b = v0 - v2, c = v1 + v3, d = v1 - v3;
  cplx<T> id = mul_i(d, DIR);  // DIR * i * d
  v0 = a + c;
  v2 = a - c;
  v1 = b + id;
  v3 = b - id;
}

template <int DIR, typename T>
CBP_HD void dft8(cplx<T>* v) {
  // even / odd split: X_k = E_k + w^k O_k, X_{k+4} = E_k - w^k O_k, w = exp(DIR 2 pi i / 8)
  cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  const T h = T(radix_consts::r2_2);
  cplx<T> w1 = {h, T(DIR) * h};    // exp(DIR i pi/4)
  cplx<T> w3 = {-h, T(DIR) * h};   // exp(DIR 3 i pi/4)
  o1 = o1 * w1;
  o2 = mul_i(o2, DIR);
  o3 = o3 * w3;
  v[0] = e0 + o0; v[4] = e0 - o0;
  v[1] = e1 + o1; v[5] = e1 - o1;
  v[2] = e2 + o2; v[6] = e2 - o2;
  v[3] = e3 + o3; v[7] = e3 - o3;
}

// Odd prime radix: with a_k = v_k + v_{R-k}, b_k = v_k - v_{R-k},
//   X_m = v_0 + sum_k a_k cos(2 pi mk/R) + DIR i sum_k b_k sin(2 pi mk/R),
//   X_{R-m} = the same with -DIR.
template <int DIR, typename T>
CBP_HD void dft3(cplx<T>* v) {
  const T c1 = T(radix_consts::c3_1), s1 = T(radix_consts::s3_1);
  cplx<T> a = v[1] + v[2], b = v[1] - v[2];
  cplx<T> A = v[0] + c1 * a;
  cplx<T> B = mul_i(s1 * b, DIR);
  v[0] = v[0] + a;
  v[1] = A + B;
  v[2] = A - B;
}

template <int DIR, typename T>
CBP_HD void dft5(cplx<T>* v) {
  const T c1 = T(radix_consts::c5_1), s1 = T(radix_consts::s5_1);
  const T c2 = T(radix_consts::c5_2), s2 = T(radix_consts::s5_2);
  cplx<T> a1 = v[1] + v[4], b1 = v[1] - v[4];
  cplx<T> a2 = v[2] + v[3], b2 = v[2] - v[3];
  cplx<T> A1 = v[0] + c1 * a1 + c2 * a2;
  cplx<T> A2 = v[0] + c2 * a1 + c1 * a2;
  cplx<T> B1 = mul_i(s1 * b1 + s2 * b2, DIR);
  cplx<T> B2 = mul_i(s2 * b1 - s1 * b2, DIR);
  v[0] = v[0] + a1 + a2;
  v[1] = A1 + B1;
  v[4] = A1 - B1;
  v[2] = A2 + B2;
  v[3] = A2 - B2;
}

template <int DIR, typename T>
CBP_HD void dft7(cplx<T>* v) {
  const T c1 = T(radix_consts::c7_1), s1 = T(radix_consts::s7_1);
  const T c2 = T(radix_consts::c7_2), s2 = T(radix_consts::s7_2);
  const T c3 = T(radix_consts::c7_3), s3 = T(radix_consts::s7_3);
  cplx<T> a1 = v[1] + v[6], b1 = v[1] - v[6];
  cplx<T> a2 = v[2] + v[5], b2 = v[2] - v[5];
  cplx<T> a3 = v[3] + v[4], b3 = v[3] - v[4];
  cplx<T> A1 = v[0] + c1 * a1 + c2 * a2 + c3 * a3;
  cplx<T> A2 = v[0] + c2 * a1 + c3 * a2 + c1 * a3;
  cplx<T> A3 = v[0] + c3 * a1 + c1 * a2 + c2 * a3;
  cplx<T> B1 = mul_i(s1 * b1 + s2 * b2 + s3 * b3, DIR);
  cplx<T> B2 = mul_i(s2 * b1 - s3 * b2 - s1 * b3, DIR);
  cplx<T> B3 = mul_i(s3 * b1 - s1 * b2 + s2 * b3, DIR);
  v[0] = v[0] + a1 + a2 + a3;
  v[1] = A1 + B1; v[6] = A1 - B1;
  v[2] = A2 + B2; v[5] = A2 - B2;
  v[3] = A3 + B3; v[4] = A3 - B3;
}

// 9 = 3 x 3: with n = 3a + b and m = c + 3d, w9^(nm) = w3^(ac) w9^(bc) w3^(bd):
// 3-point DFTs over a of x[3a + b], twiddles w9^(bc), 3-point DFTs over b.
template <int DIR, typename T>
CBP_HD void dft9(cplx<T>* v) {
  cplx<T> y[9];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    cplx<T> t[3] = {v[b], v[b + 3], v[b + 6]};
    dft3<DIR>(t);
    y[3 * b] = t[0]; y[3 * b + 1] = t[1]; y[3 * b + 2] = t[2];
  }
  const cplx<T> w1 = {T(radix_consts::c9_1), T(DIR) * T(radix_consts::s9_1)};
  const cplx<T> w2 = {T(radix_consts::c9_2), T(DIR) * T(radix_consts::s9_2)};
  const cplx<T> w4 = {T(radix_consts::c9_4), T(DIR) * T(radix_consts::s9_4)};
  y[4] = y[4] * w1;   // b = 1, c = 1
  y[5] = y[5] * w2;   // b = 1, c = 2
  y[7] = y[7] * w2;   // b = 2, c = 1
  y[8] = y[8] * w4;   // b = 2, c = 2
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx<T> t[3] = {y[c], y[3 + c], y[6 + c]};
    dft3<DIR>(t);
    v[c] = t[0]; v[c + 3] = t[1]; v[c + 6] = t[2];
  }
}

template <int R, int DIR, typename T>
CBP_HD void dft_small(cplx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 3) dft3<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 5) dft5<DIR>(v);
  else if constexpr (R == 7) dft7<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else if constexpr (R == 9) dft9<DIR>(v);
}

// ---------------------------------------------------------------- one butterfly
// 24-bit integer product (full-rate on the GPU; every index here is < 2^24).
CBP_HD int mul24(int a, int b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __mul24(a, b);
#else
  return a * b;
#endif
}

// Twiddles of a pass with radix R and stride Ns > 1 sit in a table of their
// own, entry k P + r - 1 (k < Ns, 0 < r < R) holding
// w_(Ns R)^(r k) = exp(-2 pi i r k / (Ns R)), with the odd pitch
// P = (R - 1) | 1: a butterfly reads its R - 1 twiddles at fixed offsets from
// one address, and lanes of consecutive k read from distinct LDS banks.
// The tables of a plan's passes with Ns > 1 follow each other in pass order.
CBP_HD constexpr int tw_pitch(int R) { return (R - 1) | 1; }

// Butterfly j of a radix-R pass with stride Ns (the product of the radices
// already applied) of an N-point transform at src, k = j mod Ns given: reads
// src[j + r N/R] into v, twiddles input r by w_(Ns R)^(r k) from the pass's
// table tws (TW: Ns > 1), applies the R-point DFT and returns the base
// (j - k) R + k of its outputs, which belong at base + r Ns.  The kernels run
// a pass in place: every butterfly is read before any output is written.
template <int R, int DIR, bool TW, typename T>
CBP_HD int stockham_read(const cplx<T>* src, int NR, const cplx<T>* tws, int j, int k, cplx<T>* v) {
  const cplx<T>* s = src + j;
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = s[mul24(r, NR)];
  if (TW) {
    const cplx<T>* tk = tws + mul24(k, tw_pitch(R));
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cplx<T> w = tk[r - 1];
      if (DIR > 0) w.im = -w.im;
      v[r] = v[r] * w;
    }
  }
  dft_small<R, DIR>(v);
  return mul24(j - k, R) + k;
}

// q = floor(a / b) for 0 <= a < 2^22, 1 <= b <= 2^22, from a float
// reciprocal: (a + 1/2) / b has fractional part in [1/(2b), 1 - 1/(2b)],
// further from an integer than the product's rounding error (a / b) 2^-23.
CBP_HD int fdiv_floor(int a, float rb) { return (int)(((float)a + 0.5f) * rb); }

// ---------------------------------------------------------------- plans
constexpr int FFT_MAX_PASSES = 16;

struct fft_plan {
  int N;
  int npass;
  int radix[FFT_MAX_PASSES];
  unsigned long long code;  // radix of pass s in bits [4s, 4s + 4) (device code reads this, no array index)
};

CBP_HD int plan_radix(const fft_plan& p, int s) { return (int)((p.code >> (4 * s)) & 15u); }

// Factor N into the supported radices.  `order` picks the pass order:
//   0: radix 8 first, then 4, 2, (9,) 3, 5, 7 (fewest passes);
//   1: radix 4 first, then 8, 2, (9,) 3, 5, 7;
//   2: odd radices first: 7, 5, (9,) 3, then 8, 4, 2.
// with9 takes factors 9 as one radix-9 pass before the remaining 3.
// Returns false when N has another prime factor, too many passes, or an
// unknown order.
constexpr int FFT_ORDERS = 3;

inline bool make_fft_plan(int N, fft_plan* p, int order = 0, bool with9 = false) {
  static const int orders[FFT_ORDERS][7] = {
      {8, 4, 2, 9, 3, 5, 7}, {4, 8, 2, 9, 3, 5, 7}, {7, 5, 9, 3, 8, 4, 2}};
  if (N < 1 || order < 0 || order >= FFT_ORDERS) return false;
  p->N = N;
  p->npass = 0;
  p->code = 0;
  int r = N;
  for (int t = 0; t < 7; ++t) {
    const int R = orders[order][t];
    if (R == 9 && !with9) continue;
    while (r % R == 0) {
      if (p->npass >= FFT_MAX_PASSES) return false;
      p->code |= (unsigned long long)R << (4 * p->npass);
      p->radix[p->npass++] = R;
      r /= R;
    }
  }
  return r == 1;
}

// Entries of plan p's pass twiddle tables (the passes with Ns > 1).
inline int pass_table_entries(const fft_plan& p) {
  int Ns = 1, n = 0;
  for (int s = 0; s < p.npass; ++s) {
    const int R = plan_radix(p, s);
    if (Ns > 1) n += Ns * tw_pitch(R);
    Ns *= R;
  }
  return n;
}

}  // namespace cbp
