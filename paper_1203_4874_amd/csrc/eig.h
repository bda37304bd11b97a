// Smallest eigenpair of a small Hermitian matrix (n <= 64) inside one
// workgroup: parallel cyclic Jacobi in FP64 on the rounded matrix, followed by
// Newton refinement of the smallest eigenvector against the matrix held in
// double-double.
//
// Jacobi: each round applies n/2 disjoint plane rotations chosen by the
// round-robin (circle) ordering, so one sweep of n-1 rounds (n even; an odd
// n gets a dummy index) touches every pair once.  The rotation for pair
// (p, q) with a_pq = |a_pq| e^{i phi} is
//   U = [[c, s e^{i phi}], [-s e^{-i phi}, c]]   (rows/cols p, q),
// with t = sign(tau) / (|tau| + sqrt(1 + tau^2)), tau = (a_qq - a_pp) / (2 |a_pq|),
// c = 1/sqrt(1+t^2), s = t c; it zeroes a_pq of U^H A U (Rutishauser's form
// of the classical Jacobi rotation, applied to the phase-rotated pair).
// Sweeps stop when the off-diagonal energy falls below 1e-28 of the diagonal
// energy.
//
// Refinement: with (lam_k, v_k) from Jacobi and x the current vector,
//   r = G x - mu x  (mu = x^H G x),  both in double-double,
//   x <- x - sum_{k != min} v_k (v_k^H r) / (lam_k - mu),  x <- x / ||x||.
// This is a Newton step on the eigenvector equation, preconditioned by the
// FP64 eigen-decomposition; each step shrinks the error by about
// eps ||G|| / (lam_1 - lam_0).
#pragma once

#include "common.h"

namespace cbp {

constexpr int EIG_NT = 512;
constexpr int EIG_MAXN = 64;
constexpr int EIG_MAX_SWEEPS = 20;
constexpr int EIG_REFINE = 2;

// LDS working set of the solver.  Sizes: A, V n*n; vectors n.
struct eig_ws {
  c64* A;
  c64* V;
  double* lam;
  int* pp;      // pair slots: p, q, c, s e^{i phi}
  int* qq;
  double* cs;
  c64* se;
  c64* x;
  c64* r;
  c64* beta;
  double* red;  // EIG_NT doubles
  int* misc;    // 4 ints
};

__host__ __device__ inline size_t eig_lds_bytes(int n) {
  return (size_t)2 * n * n * sizeof(c64) + (size_t)n * (2 * sizeof(double) + 2 * sizeof(int) + 4 * sizeof(c64)) +
         EIG_NT * sizeof(double) + 4 * sizeof(int) + 64;
}

// Carve the working set out of a dynamic LDS block (16-byte aligned pieces).
__device__ inline eig_ws eig_carve(char* base, int n) {
  eig_ws w;
  char* p = base;
  w.A = (c64*)p; p += (size_t)n * n * sizeof(c64);
  w.V = (c64*)p; p += (size_t)n * n * sizeof(c64);
  w.se = (c64*)p; p += n * sizeof(c64);
  w.x = (c64*)p; p += n * sizeof(c64);
  w.r = (c64*)p; p += n * sizeof(c64);
  w.beta = (c64*)p; p += n * sizeof(c64);
  w.lam = (double*)p; p += n * sizeof(double);
  w.cs = (double*)p; p += n * sizeof(double);
  w.red = (double*)p; p += EIG_NT * sizeof(double);
  w.pp = (int*)p; p += n * sizeof(int);
  w.qq = (int*)p; p += n * sizeof(int);
  w.misc = (int*)p;
  return w;
}

// Deterministic block sum over EIG_NT threads (fixed tree).
__device__ inline double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = EIG_NT / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// dd sum over the 64 lanes of wave 0 (xor butterfly; dd_add is commutative,
// so every lane ends with the same value).  Only wave 0 may call it.
__device__ inline dd wave_sum_dd(dd v) {
  for (int m = 32; m > 0; m >>= 1) {
    dd o;
    o.hi = __shfl_xor(v.hi, m, 64);
    o.lo = __shfl_xor(v.lo, m, 64);
    v = dd_add(v, o);
  }
  return v;
}

__device__ inline double wave_sum(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Rotation of pair slot k = (p, q) from the current A.  The 2 x 2 unitary on
// (p, q) is [[c, se], [-conj(se), c]] with se = s e^{i phi}; stored as (c, se).
__device__ inline void jacobi_rotation(eig_ws& w, int n, int k, int p, int q) {
  w.pp[k] = p;
  w.qq[k] = q;
  const c64 apq = w.A[p * n + q];
  const double app = w.A[p * n + p].re, aqq = w.A[q * n + q].re;
  const double mag = hypot(apq.re, apq.im);
  if (!(mag > 1e-300)) {
    w.cs[k] = 1.0;
    w.se[k] = {0.0, 0.0};
    return;
  }
  const double tau = (aqq - app) / (2.0 * mag);
  double t;
  if (fabs(tau) < 1e150) t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  else t = 0.5 / tau;
  const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
  w.cs[k] = c;
  w.se[k] = {sn * apq.re / mag, sn * apq.im / mag};
}

// Jacobi on w.A (n x n, Hermitian) -> eigenvalues in w.lam, eigenvectors in
// the columns of w.V.  Each round: rotations of the round's pairs, then
// A <- U^H A (row pairs), then A <- A U and V <- V U (column pairs); every
// task owns the two entries it rewrites, so the updates are in place.
// Returns the number of sweeps run.
__device__ inline int jacobi_eig(eig_ws& w, int n) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += EIG_NT) {
    const int i = e / n, j = e - i * n;
    w.V[e] = {i == j ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  const int nn = n + (n & 1);
  const int np = nn / 2;
  int sweep = 0;
  for (; sweep < EIG_MAX_SWEEPS; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += EIG_NT) {
      const int i = e / n, j = e - i * n;
      const double v = norm2(w.A[e]);
      if (i == j) dia += v; else off += v;
    }
    off = block_sum(off, w.red);
    dia = block_sum(dia, w.red);
    if (!(off > 1e-28 * dia)) break;
    for (int round = 0; round < nn - 1; ++round) {
      if (tid < np) {
        int p, q;
        if (tid == 0) { p = round; q = nn - 1; }
        else { p = (round + tid) % (nn - 1); q = (round - tid + (nn - 1)) % (nn - 1); }
        if (p < n && q < n) jacobi_rotation(w, n, tid, p, q);
        else { w.pp[tid] = -1; w.qq[tid] = -1; }
      }
      __syncthreads();
      // rows: A[p][j], A[q][j]
      for (int t = tid; t < np * n; t += EIG_NT) {
        const int k = t / n, j = t - k * n;
        const int p = w.pp[k];
        if (p < 0) continue;
        const int q = w.qq[k];
        const double c = w.cs[k];
        const c64 se = w.se[k];
        const c64 ap = w.A[p * n + j], aq = w.A[q * n + j];
        // (U^H A)[p][j] = c a_p - se a_q ;  (U^H A)[q][j] = conj(se) a_p + c a_q
        w.A[p * n + j] = c * ap - se * aq;
        w.A[q * n + j] = cmulc(se, ap) + c * aq;
      }
      __syncthreads();
      // columns of A and of V: X[i][p], X[i][q]
      for (int t = tid; t < 2 * np * n; t += EIG_NT) {
        const int half = t >= np * n;
        const int tt = half ? t - np * n : t;
        const int k = tt / n, i = tt - k * n;
        const int p = w.pp[k];
        if (p < 0) continue;
        const int q = w.qq[k];
        const double c = w.cs[k];
        const c64 se = w.se[k];
        c64* X = half ? w.V : w.A;
        const c64 xp = X[i * n + p], xq = X[i * n + q];
        // (X U)[i][p] = c x_p - conj(se) x_q ;  (X U)[i][q] = se x_p + c x_q
        X[i * n + p] = c * xp - conj(se) * xq;
        X[i * n + q] = se * xp + c * xq;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += EIG_NT) w.lam[i] = w.A[i * n + i].re;
  __syncthreads();
  return sweep;
}

// Index of the smallest eigenvalue and the second smallest value (wave 0
// computes, result broadcast through LDS).
__device__ inline int eig_argmin(eig_ws& w, int n, double* second) {
  if (threadIdx.x == 0) {
    int im = 0;
    for (int i = 1; i < n; ++i) if (w.lam[i] < w.lam[im]) im = i;
    double s2 = 1.7976931348623157e308;
    for (int i = 0; i < n; ++i) if (i != im && w.lam[i] < s2) s2 = w.lam[i];
    w.misc[0] = im;
    w.red[0] = (n > 1) ? s2 : w.lam[im];
  }
  __syncthreads();
  const int im = w.misc[0];
  *second = w.red[0];
  __syncthreads();
  return im;
}

// Newton refinement of the eigenvector for eigenvalue index imin against the
// double-double matrix given by acc.get(i, j) (a cdd).  Leaves the unit
// vector in w.x and returns mu = x^H G x (as dd).
template <class Acc>
__device__ inline dd eig_refine(eig_ws& w, const Acc& acc, int n, int imin) {
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += EIG_NT) w.x[i] = w.V[i * n + imin];
  __syncthreads();
  dd mu = {0.0, 0.0};
  for (int it = 0; it <= EIG_REFINE; ++it) {
    // y = G x (dd) and mu = x^H y (dd), wave 0 (n <= 64 lanes)
    dd yre = {0.0, 0.0}, yim = {0.0, 0.0};
    c64 xi = {0.0, 0.0};
    if (tid < 64) {
      if (tid < n) {
        xi = w.x[tid];
        dot2 ar, ai;
        ar.init();
        ai.init();
        for (int j = 0; j < n; ++j) {
          const cdd g = acc.get(tid, j);
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
      mu = wave_sum_dd(t.result());
      if (tid < n) {
        dot2 qr, qi;
        qr.init(); qi.init();
        qr.add_dd(yre); qr.add_prod(-mu.hi, xi.re); qr.add(-mu.lo * xi.re);
        qi.add_dd(yim); qi.add_prod(-mu.hi, xi.im); qi.add(-mu.lo * xi.im);
        const dd rr = qr.result(), ri = qi.result();
        w.r[tid] = {dd_val(rr), dd_val(ri)};
      }
      if (tid == 0) { w.red[0] = mu.hi; w.red[1] = mu.lo; }
    }
    __syncthreads();
    mu.hi = w.red[0];
    mu.lo = w.red[1];
    if (it == EIG_REFINE) break;
    // beta_k = v_k^H r / (lam_k - mu), k != imin
    if (tid < n) {
      c64 s = {0.0, 0.0};
      for (int i = 0; i < n; ++i) s = s + cmulc(w.V[i * n + tid], w.r[i]);
      const double den = w.lam[tid] - mu.hi;
      c64 b = {0.0, 0.0};
      if (tid != imin && fabs(den) > 0.0) b = {s.re / den, s.im / den};
      w.beta[tid] = b;
    }
    __syncthreads();
    // x <- x - V beta, then normalise (wave 0)
    if (tid < 64) {
      c64 xn = {0.0, 0.0};
      if (tid < n) {
        c64 d = {0.0, 0.0};
        for (int k = 0; k < n; ++k) d = d + w.V[tid * n + k] * w.beta[k];
        xn = w.x[tid] - d;
      }
      const double nrm = sqrt(wave_sum(norm2(xn)));
      if (tid < n && nrm > 0.0) w.x[tid] = {xn.re / nrm, xn.im / nrm};
    }
    __syncthreads();
  }
  return mu;
}

}  // namespace cbp
