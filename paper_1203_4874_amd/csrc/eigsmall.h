// Smallest eigenpair of a small Hermitian matrix (n <= 64) in one wave.
//
//  1. Householder reduction of the FP64 matrix to a Hermitian tridiagonal
//     Q^H G Q, then a diagonal unitary D that makes it real: T = D^H Q^H G Q D
//     with diagonal a_k and off-diagonal b_k = |e_k| >= 0 (Golub & Van Loan,
//     "Matrix Computations", Sec. 8.3.1).
//  2. The two smallest eigenvalues of T by Sturm-count multisection: the
//     number of negative pivots of the LDL^T factorisation of T - s I is the
//     number of eigenvalues below s (Sylvester's law of inertia); 32 lanes
//     each probe one point of the current bracket per round, 12 rounds.
//  3. sigma = lam0 - max(1e-3 (lam1 - lam0), 16 n eps ||T||), so that
//     G - sigma I is positive definite with its smallest eigenvalue well
//     separated; its inverse M by Gauss-Jordan elimination (no pivoting is
//     needed for a positive definite matrix).
//  4. Shifted inverse iteration x <- M x / ||M x|| (error shrinks by
//     (lam0 - sigma) / (lam1 - sigma) per step).
//  5. Newton refinement against G held in double-double:
//       r = G x - mu x (mu = x^H G x, both double-double),
//       x <- (x - M r) / ||x - M r||,
//     until ||M r|| < 1e-15; M r approximates the exact Newton correction
//     sum_k v_k (v_k^H r) / (lam_k - mu) with relative error
//     (mu - sigma) / (lam_k - sigma) ~ 1e-3.
// Everything runs in one wave of 64 lanes; matrices live in LDS.
#pragma once

#include "common.h"

namespace cbp {

constexpr int SMALL_NT = 64;
constexpr int SMALL_REFINE_MAX = 4;
constexpr int SMALL_INVIT = 5;
constexpr int SMALL_BISECT_ROUNDS = 12;

struct small_ws {
  c64* A;       // n*n: Householder work matrix, then (G - sigma I)^{-1}
  double* a;    // n: diagonal of T
  double* b;    // n: off-diagonal of T, b[k] = T[k+1][k]
  c64* e;       // n: complex off-diagonal before the phase fix
  c64* x;       // n: eigenvector estimate
  c64* y;       // n: scratch vector
  c64* r;       // n: scratch vector
  double* red;  // 8 doubles
};

__host__ __device__ inline size_t small_lds_bytes(int n) {
  return (size_t)n * n * sizeof(c64) + (size_t)n * (2 * sizeof(double) + 4 * sizeof(c64)) + 8 * sizeof(double) + 64;
}

__device__ inline small_ws small_carve(char* base, int n) {
  small_ws w;
  char* p = base;
  w.A = (c64*)p; p += (size_t)n * n * sizeof(c64);
  w.e = (c64*)p; p += n * sizeof(c64);
  w.x = (c64*)p; p += n * sizeof(c64);
  w.y = (c64*)p; p += n * sizeof(c64);
  w.r = (c64*)p; p += n * sizeof(c64);
  w.a = (double*)p; p += n * sizeof(double);
  w.b = (double*)p; p += n * sizeof(double);
  w.red = (double*)p;
  return w;
}

// Reciprocal and reciprocal square root: hardware estimate + two Newton steps.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

__device__ inline double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// (e / n, e % n) without an integer division (float estimate, corrected).
__device__ inline void split_index(int e, int n, float rn, int& i, int& j) {
  i = (int)((float)e * rn);
  j = e - i * n;
  if (j >= n) { ++i; j -= n; }
  else if (j < 0) { --i; j += n; }
}

// Wave-wide reductions (xor butterflies: every lane gets the same value).
__device__ inline double wsum(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ inline double wmin(double v) {
  for (int m = 32; m > 0; m >>= 1) v = fmin(v, __shfl_xor(v, m, 64));
  return v;
}
__device__ inline double wmax(double v) {
  for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}
__device__ inline c64 wsum_c(c64 v) { return {wsum(v.re), wsum(v.im)}; }
__device__ inline c64 shfl_c(c64 v, int src) { return {__shfl(v.re, src, 64), __shfl(v.im, src, 64)}; }

__device__ inline dd wsum_dd(dd v) {
  for (int m = 32; m > 0; m >>= 1) {
    dd o;
    o.hi = __shfl_xor(v.hi, m, 64);
    o.lo = __shfl_xor(v.lo, m, 64);
    v = dd_add(v, o);
  }
  return v;
}

// 1. Householder tridiagonalisation of w.A (n x n Hermitian, destroyed);
//    leaves T in w.a, w.b.
__device__ inline void small_tridiag(small_ws& w, int n) {
  const int l = threadIdx.x;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;       // length of the column below the diagonal
    const int o = k + 1;
    c64 xl = {0.0, 0.0};
    if (l < m) xl = conj(w.A[k * n + o + l]);   // A[o+l][k] = conj(A[k][o+l])
    const double s2 = wsum(norm2(xl));
    const double tail = wsum(l >= 1 ? norm2(xl) : 0.0);
    const c64 x0 = shfl_c(xl, 0);
    if (!(tail > 0.0)) {                         // column already reduced
      if (l == 0) w.e[k] = x0;
      __syncthreads();
      continue;
    }
    const double nx = s2 * rsq_nr(s2);          // ||x||
    const double ax0 = sqrt(norm2(x0));
    const c64 ph = ax0 > 0.0 ? c64{x0.re / ax0, x0.im / ax0} : c64{1.0, 0.0};
    const c64 alpha = {-ph.re * nx, -ph.im * nx};
    // v = sqrt(2) u / ||u||, u = x - alpha e_0, ||u||^2 = 2 ||x|| (||x|| + |x_0|)
    const double sc = rsq_nr(nx * (nx + ax0));
    c64 vl = {0.0, 0.0};
    if (l < m) {
      const c64 ul = (l == 0) ? c64{xl.re - alpha.re, xl.im - alpha.im} : xl;
      vl = {ul.re * sc, ul.im * sc};
      w.x[l] = vl;
    }
    __syncthreads();
    // p = A' v with A' the trailing m x m block (read by columns: A'[l][j] = conj(A'[j][l]))
    c64 pl = {0.0, 0.0};
    if (l < m)
      for (int j = 0; j < m; ++j) pl = pl + cmulc(w.A[(o + j) * n + o + l], w.x[j]);
    const double K = 0.5 * wsum(l < m ? (vl.re * pl.re + vl.im * pl.im) : 0.0);  // Re(v^H p) / 2
    const c64 wl = {pl.re - K * vl.re, pl.im - K * vl.im};
    if (l < m) w.y[l] = wl;
    __syncthreads();
    // A' -= v w^H + w v^H   (lane l rewrites column l)
    if (l < m) {
      const c64 cw = conj(wl), cv = conj(vl);
      for (int j = 0; j < m; ++j) {
        const c64 vj = w.x[j], wj = w.y[j];
        const size_t id = (size_t)(o + j) * n + o + l;
        w.A[id] = w.A[id] - vj * cw - wj * cv;
      }
    }
    if (l == 0) w.e[k] = alpha;
    __syncthreads();
  }
  if (l < n) w.a[l] = w.A[l * n + l].re;
  if (l == 0 && n >= 2) w.e[n - 2] = w.A[(n - 1) * n + n - 2];
  __syncthreads();
  if (l < n - 1) w.b[l] = sqrt(norm2(w.e[l]));
  if (l == n - 1) w.b[l] = 0.0;
  __syncthreads();
}

// Number of eigenvalues of T below s (Sturm count).
__device__ inline int sturm_count(const double* a, const double* b, int n, double s, double pivmin) {
  double q = a[0] - s;
  int c = q < 0.0;
  for (int k = 1; k < n; ++k) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = a[k] - s - b[k - 1] * b[k - 1] * rcp_nr(q);
    c += q < 0.0;
  }
  return c;
}

// 2. Two smallest eigenvalues of T (n >= 2; lanes 0-31 bracket lam0, 32-63 lam1).
__device__ inline void small_bisect(small_ws& w, int n, double* lam0, double* lam1, double* tnorm) {
  const int l = threadIdx.x;
  double glo = 1.7976931348623157e308, ghi = -1.7976931348623157e308, bmax = 0.0;
  if (l < n) {
    const double bl = l > 0 ? w.b[l - 1] : 0.0, br = w.b[l];
    glo = w.a[l] - bl - br;
    ghi = w.a[l] + bl + br;
    bmax = br;
  }
  glo = wmin(glo);
  ghi = wmax(ghi);
  bmax = wmax(bmax);
  const double tn = fmax(fabs(glo), fabs(ghi));
  const double pivmin = fmax(bmax * bmax, 1e-280) * 1e-290 + 1e-300;
  const int g = l >> 5, j = l & 31;
  const int target = g + 1;                       // need count >= target
  double lo = glo - 2.2e-16 * tn - 1e-300, hi = ghi + 2.2e-16 * tn + 1e-300;
  for (int it = 0; it < SMALL_BISECT_ROUNDS; ++it) {
    const double h = (hi - lo) * (1.0 / 33.0);
    const double s = lo + h * (double)(j + 1);
    const bool hit = sturm_count(w.a, w.b, n, s, pivmin) >= target;
    const unsigned long long mask = __ballot(hit);
    const unsigned int gm = (unsigned int)(mask >> (32 * g));
    const int js = gm ? __builtin_ctz(gm) : 32;   // first probe at or above the eigenvalue
    const double nlo = js == 0 ? lo : lo + h * (double)js;
    const double nhi = js == 32 ? hi : lo + h * (double)(js + 1);
    lo = nlo;
    hi = nhi;
  }
  const double mid = 0.5 * (lo + hi);
  *lam0 = __shfl(mid, 0, 64);
  *lam1 = n >= 2 ? __shfl(mid, 32, 64) : *lam0;
  *tnorm = tn;
}

// 3. w.A <- (B)^{-1} for the Hermitian positive definite B already in w.A
//    (Gauss-Jordan, no pivoting; row and column k are staged in w.y / w.r).
__device__ inline void small_gj_inverse(small_ws& w, int n) {
  const int l = threadIdx.x;
  const float rn = 1.0f / (float)n;
  for (int k = 0; k < n; ++k) {
    if (l < n) {
      w.y[l] = w.A[l * n + k];
      w.r[l] = w.A[k * n + l];
    }
    __syncthreads();
    const double ip = rcp_nr(w.r[k].re);
    for (int e = l; e < n * n; e += SMALL_NT) {
      int i, jj;
      split_index(e, n, rn, i, jj);
      c64 v;
      if (i == k && jj == k) v = {ip, 0.0};
      else if (i == k) v = ip * w.r[jj];
      else if (jj == k) v = -ip * w.y[i];
      else v = w.A[e] - ip * (w.y[i] * w.r[jj]);
      w.A[e] = v;
    }
    __syncthreads();
  }
}

// y = M x with M = w.A Hermitian (lane l reads column l: M[l][j] = conj(M[j][l])).
__device__ inline c64 small_matvec(const small_ws& w, int n, const c64* x) {
  const int l = threadIdx.x;
  c64 s = {0.0, 0.0};
  if (l < n)
    for (int j = 0; j < n; ++j) s = s + cmulc(w.A[j * n + l], x[j]);
  return s;
}

// The whole solver.  acc.get(i, j) gives G in double-double; G's rounded
// value must already be in w.A.  Returns mu = x^H G x (dd); x is left in w.x
// (unit norm).  *lam1 receives the second smallest eigenvalue of the FP64
// matrix and *steps the number of refinement steps.
template <class Acc>
__device__ inline dd small_eig(small_ws& w, const Acc& acc, int n, double* lam1, int* steps) {
  const int l = threadIdx.x;
  if (n == 1) {
    if (l == 0) w.x[0] = {1.0, 0.0};
    __syncthreads();
    *lam1 = dd_val(acc.get(0, 0).re);
    *steps = 0;
    return acc.get(0, 0).re;
  }
  small_tridiag(w, n);
  double l0, l1, tn;
  small_bisect(w, n, &l0, &l1, &tn);
  *lam1 = l1;
  const double shift = fmax(1e-3 * (l1 - l0), 16.0 * n * 2.2e-16 * tn);
  const double sigma = l0 - shift;
  // B = G - sigma I (rounded G), inverted in place
  for (int e = l; e < n * n; e += SMALL_NT) {
    const int i = e / n, jj = e - i * n;
    const cdd g = acc.get(i, jj);
    w.A[e] = {g.re.hi - (i == jj ? sigma : 0.0), g.im.hi};
  }
  __syncthreads();
  small_gj_inverse(w, n);
  // inverse iteration from a fixed, generic start vector
  if (l < n) w.x[l] = {1.0 + 0.6180339887 * (double)l, 0.5 - 0.4142135624 * (double)((l * 7) % 5)};
  __syncthreads();
  for (int it = 0; it < SMALL_INVIT; ++it) {
    const c64 y = small_matvec(w, n, w.x);
    const double nr = sqrt(wsum(l < n ? norm2(y) : 0.0));
    __syncthreads();
    if (l < n) w.x[l] = {y.re / nr, y.im / nr};
    __syncthreads();
  }
  // Newton refinement against the double-double matrix
  dd mu = {0.0, 0.0};
  int it = 0;
  bool done = false;
  for (;; ++it) {
    dd yre = {0.0, 0.0}, yim = {0.0, 0.0};
    c64 xi = {0.0, 0.0};
    if (l < n) {
      xi = w.x[l];
      dot2 ar, ai;
      ar.init();
      ai.init();
      for (int j = 0; j < n; ++j) {
        const cdd g = acc.get(l, j);
        const c64 xj = w.x[j];
        ar.add_prod(g.re.hi, xj.re); ar.add(g.re.lo * xj.re);
        ar.add_prod(-g.im.hi, xj.im); ar.add(-g.im.lo * xj.im);
        ai.add_prod(g.re.hi, xj.im); ai.add(g.re.lo * xj.im);
        ai.add_prod(g.im.hi, xj.re); ai.add(g.im.lo * xj.re);
      }
      yre = ar.result();
      yim = ai.result();
    }
    dot2 t;
    t.init();
    t.add_prod(xi.re, yre.hi); t.add(xi.re * yre.lo);
    t.add_prod(xi.im, yim.hi); t.add(xi.im * yim.lo);
    mu = wsum_dd(t.result());
    if (done || it == SMALL_REFINE_MAX) break;
    if (l < n) {
      dot2 qr, qi;
      qr.init(); qi.init();
      qr.add_dd(yre); qr.add_prod(-mu.hi, xi.re); qr.add(-mu.lo * xi.re);
      qi.add_dd(yim); qi.add_prod(-mu.hi, xi.im); qi.add(-mu.lo * xi.im);
      w.r[l] = {dd_val(qr.result()), dd_val(qi.result())};
    }
    __syncthreads();
    const c64 d = small_matvec(w, n, w.r);
    const c64 xn = l < n ? xi - d : c64{0.0, 0.0};
    const double nrm = sqrt(wsum(norm2(xn)));
    const double dn = sqrt(wsum(l < n ? norm2(d) : 0.0));
    __syncthreads();
    if (l < n) w.x[l] = {xn.re / nrm, xn.im / nrm};
    __syncthreads();
    done = !(dn > 1e-15);
  }
  *steps = it;
  return mu;
}

}  // namespace cbp
