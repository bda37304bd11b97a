// Shared device/host helpers of the CBP library: complex values, double-double
// arithmetic (error-free transformations), error codes and launch checks.
//
// Double-double arithmetic follows the error-free transformations of Knuth
// (TwoSum), Dekker (FastTwoSum) and the FMA-based TwoProduct, and the
// compensated dot product "Dot2" of Ogita, Rump and Oishi (SIAM J. Sci.
// Comput. 26(6), 2005): a sum of products accumulated as if in twice the
// working precision.  FMA contraction is disabled inside these helpers so the
// compiler cannot fuse the operations whose rounding errors they capture.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define CBP_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define CBP_HD inline
#endif

namespace cbp {

// ---------------------------------------------------------------- complex
template <typename T>
struct cplx {
  T re, im;
};

template <typename T> CBP_HD cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T> CBP_HD cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> CBP_HD cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> CBP_HD cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> CBP_HD cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> CBP_HD cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// multiply by +i (s = +1) or -i (s = -1)
template <typename T> CBP_HD cplx<T> mul_i(cplx<T> a, int s) { return s > 0 ? cplx<T>{-a.im, a.re} : cplx<T>{a.im, -a.re}; }
template <typename T> CBP_HD T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
// conj(a) * b
template <typename T> CBP_HD cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T, typename U> CBP_HD cplx<T> cast(cplx<U> a) { return {T(a.re), T(a.im)}; }

using c64 = cplx<double>;
using c32 = cplx<float>;

// ---------------------------------------------------------------- double-double
struct dd {
  double hi, lo;
};

CBP_HD void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

CBP_HD void fast_two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  e = b - (s - a);
}

CBP_HD void two_prod(double a, double b, double& p, double& e) {
#pragma clang fp contract(off)
  p = a * b;
  e = fma(a, b, -p);
}

CBP_HD dd dd_add(dd x, dd y) {
#pragma clang fp contract(off)
  double s, e;
  two_sum(x.hi, y.hi, s, e);
  e += x.lo + y.lo;
  dd r;
  fast_two_sum(s, e, r.hi, r.lo);
  return r;
}

CBP_HD dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
CBP_HD double dd_val(dd x) { return x.hi + x.lo; }

// Dot2 accumulator: p + s carries the running sum of exact products.
struct dot2 {
  double p, s;
  CBP_HD void init() { p = 0.0; s = 0.0; }
  CBP_HD void add_prod(double a, double b) {
#pragma clang fp contract(off)
    double h, r, q;
    two_prod(a, b, h, r);
    two_sum(p, h, p, q);
    s += q + r;
  }
  CBP_HD void add(double a) {
#pragma clang fp contract(off)
    double q;
    two_sum(p, a, p, q);
    s += q;
  }
  CBP_HD void add_dd(dd a) {
#pragma clang fp contract(off)
    double q;
    two_sum(p, a.hi, p, q);
    s += q + a.lo;
  }
  CBP_HD dd result() const {
    dd r;
    fast_two_sum(p, s, r.hi, r.lo);
    return r;
  }
};

// complex double-double
struct cdd {
  dd re, im;
};

CBP_HD cdd cdd_add(cdd a, cdd b) { return {dd_add(a.re, b.re), dd_add(a.im, b.im)}; }
CBP_HD cdd cdd_conj(cdd a) { return {a.re, dd_neg(a.im)}; }
CBP_HD cdd cdd_neg(cdd a) { return {dd_neg(a.re), dd_neg(a.im)}; }
CBP_HD c64 cdd_val(cdd a) { return {dd_val(a.re), dd_val(a.im)}; }

// ---------------------------------------------------------------- small DFT constants
// cos and sin of 2 pi k / R for the odd radices (values of the circular
// functions at rational multiples of pi, to 20 significant digits).
struct radix_consts {
  static constexpr double c3_1 = -0.5;
  static constexpr double s3_1 = 0.86602540378443864676;   // sqrt(3)/2
  static constexpr double c5_1 = 0.30901699437494742410;   // (sqrt(5)-1)/4
  static constexpr double s5_1 = 0.95105651629515357212;
  static constexpr double c5_2 = -0.80901699437494742410;  // -(sqrt(5)+1)/4
  static constexpr double s5_2 = 0.58778525229247312917;
  static constexpr double c7_1 = 0.62348980185873353053;
  static constexpr double s7_1 = 0.78183148246802980871;
  static constexpr double c7_2 = -0.22252093395631440429;
  static constexpr double s7_2 = 0.97492791218182360702;
  static constexpr double c7_3 = -0.90096886790241912624;
  static constexpr double s7_3 = 0.43388373911755812048;
  static constexpr double c9_1 = 0.76604444311897803520;   // cos / sin (2 pi k / 9), k = 1, 2, 4
  static constexpr double s9_1 = 0.64278760968653932632;
  static constexpr double c9_2 = 0.17364817766693034885;
  static constexpr double s9_2 = 0.98480775301220805937;
  static constexpr double c9_4 = -0.93969262078590838405;
  static constexpr double s9_4 = 0.34202014332566873304;
  static constexpr double r2_2 = 0.70710678118654752440;   // sqrt(2)/2
};

}  // namespace cbp
