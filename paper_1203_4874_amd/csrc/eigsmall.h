// Smallest eigenpair of a small Hermitian matrix (n <= 64) in one wave.
//
//  1. Householder reduction of the FP64 matrix to a Hermitian tridiagonal
//     (Golub & Van Loan, "Matrix Computations", Sec. 8.3.1); with a diagonal
//     unitary it becomes the real tridiagonal T (diagonal a_k, off-diagonal
//     b_k = |e_k|), which has the same eigenvalues.
//  2. The smallest eigenvalue of T by Sturm-count multisection: the number of
//     negative pivots of the LDL^T factorisation of T - s I is the number of
//     eigenvalues below s (Sylvester's law of inertia).  64 probes per round,
//     8 rounds, leave a bracket [lo, hi] of width ~6e-15 ||T||.
//  3. sigma = lo - 16 n eps ||T|| < lam0, so T - sigma I is positive
//     definite with its smallest eigenvalue well separated from the rest; its
//     LDL^T factors (d_k > 0) give X = (T - sigma I)^{-1} explicitly (one
//     column per lane).  Inverse iteration runs on T (y <- X y) and
//     x = W y with W = Q D: the Householder reflectors (kept in the reduced
//     matrix's strictly lower part) applied one by one, after the diagonal
//     unitary D that makes the tridiagonal real.
//  4. Newton refinement against G held in double-double:
//       r = G x - mu x (mu = x^H G x, both double-double),
//       x <- (x - M r) / ||x - M r||,  M = W X W^H,
//     until the change of direction (the correction's part orthogonal to x)
//     is below 4e-15; M r approximates the exact Newton
//     step sum_k v_k (v_k^H r) / (lam_k - mu) with relative error
//     (mu - sigma) / (lam_k - sigma).
//
// One lane holds one vector entry (n <= 64); matrices live in LDS.  Wave
// reductions use DPP lane permutations (quad_perm, half-row and row mirrors,
// row broadcasts of lanes 15 and 31) and a read of lane 63, which keeps them
// in the vector ALU instead of the LDS permute path.  LDS loads of a loop are
// issued in batches before their uses so their latency overlaps.
#pragma once

#include "common.h"

namespace cbp {

constexpr int SMALL_NT = 64;
constexpr int SMALL_REFINE_MAX = 4;
constexpr int SMALL_INVIT = 3;
constexpr int SMALL_BISECT_ROUNDS = 8;

struct small_ws {
  c64* A;       // n*n: matrix being reduced; afterwards the reflectors below the diagonal
  c64* e;       // n: complex off-diagonal of the Hermitian tridiagonal
  c64* w;       // n: scratch (Householder vector; then the LDL^T factors {1/d_k, l_k})
  c64* u;       // n: scratch (Householder w; then the right-hand side of a tridiagonal solve)
  c64* x;       // n: result vector
  double* a;    // n: diagonal of T
  double* b;    // n: off-diagonal of T, b[k] = T[k+1][k]
  dd* part;     // 64 x 2: partial double-double row sums of the refinement's product (ng n <= 64 lanes)
  c64* W;       // with a caller half: n x (n+1) entries, the solver keeping X in the second half and
                //   callers up to n^2 doubles in the first half across a solve; else X alone
  double* X;    // n x n: (T - sigma I)^{-1}
};

// LDS of a solve of order n; caller_half: the W region also holds the
// caller's n^2 doubles (the scale solve's coupling block), else only X (a
// smaller footprint, so that the sample solves fit on a CU beside the FFT
// passes' workgroups).
__host__ __device__ inline size_t small_lds_bytes(int n, bool caller_half = true) {
  return (size_t)n * n * sizeof(c64) + (size_t)n * (4 * sizeof(c64) + 2 * sizeof(double)) +
         (size_t)SMALL_NT * 2 * sizeof(dd) +
         (caller_half ? (size_t)n * (n + 1) * sizeof(c64) : (size_t)n * n * sizeof(double)) + 64;
}

__device__ inline small_ws small_carve(char* base, int n, bool caller_half = true) {
  small_ws s;
  char* p = base;
  s.A = (c64*)p; p += (size_t)n * n * sizeof(c64);
  s.e = (c64*)p; p += n * sizeof(c64);
  s.w = (c64*)p; p += n * sizeof(c64);
  s.u = (c64*)p; p += n * sizeof(c64);
  s.x = (c64*)p; p += n * sizeof(c64);
  s.a = (double*)p; p += n * sizeof(double);
  s.b = (double*)p; p += n * sizeof(double);
  s.part = (dd*)p; p += (size_t)SMALL_NT * 2 * sizeof(dd);
  s.W = (c64*)p;
  s.X = caller_half ? (double*)p + (size_t)n * n : (double*)p;
  return s;
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

// ---------------------------------------------------------------- wave primitives
template <int CTRL, int ROWMASK = 0xf>
__device__ inline double dpp_d(double v, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ inline double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Lane permutation with zero fill: lanes whose source lies outside the wave
// read 0 (bound control), so no prior value of the destination is needed.
template <int CTRL>
__device__ inline double dpp_z(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes (fixed order; the result is wave-uniform).  Within
// each row of 16 lanes: quad permutations and row mirrors; then lane 15 of
// each row is added into the next row and lane 31 into rows 2 and 3, so lane
// 63 ends with ((r3 + r2) + (r1 + r0)) of the row sums r0..r3 (other lanes
// may hold partial or doubled sums and are not read).
__device__ inline double wsum(double v) {
  v += dpp_z<0xB1>(v);     // quad_perm [1,0,3,2]
  v += dpp_z<0x4E>(v);     // quad_perm [2,3,0,1]
  v += dpp_z<0x141>(v);    // row_half_mirror
  v += dpp_z<0x140>(v);    // row_mirror
  v += dpp_z<0x142>(v);    // row_bcast:15
  v += dpp_z<0x143>(v);    // row_bcast:31
  return readlane_d(v, 63);
}

__device__ inline double wmin(double v) {
  const double inf = __builtin_inf();
  v = fmin(v, dpp_d<0xB1>(v, inf));
  v = fmin(v, dpp_d<0x4E>(v, inf));
  v = fmin(v, dpp_d<0x141>(v, inf));
  v = fmin(v, dpp_d<0x140>(v, inf));
  v = fmin(v, dpp_d<0x142, 0xa>(v, inf));
  v = fmin(v, dpp_d<0x143, 0xc>(v, inf));
  return readlane_d(v, 63);
}

__device__ inline double wmax(double v) { return -wmin(-v); }

__device__ inline c64 wsum_c(c64 v) {
  v.re += dpp_z<0xB1>(v.re);  v.im += dpp_z<0xB1>(v.im);
  v.re += dpp_z<0x4E>(v.re);  v.im += dpp_z<0x4E>(v.im);
  v.re += dpp_z<0x141>(v.re); v.im += dpp_z<0x141>(v.im);
  v.re += dpp_z<0x140>(v.re); v.im += dpp_z<0x140>(v.im);
  v.re += dpp_z<0x142>(v.re); v.im += dpp_z<0x142>(v.im);
  v.re += dpp_z<0x143>(v.re); v.im += dpp_z<0x143>(v.im);
  return {readlane_d(v.re, 63), readlane_d(v.im, 63)};
}

// The same sum when only lanes 0..31 can be nonzero: lane 31 ends with
// r1 + r0.
__device__ inline c64 wsum_c32(c64 v) {
  v.re += dpp_z<0xB1>(v.re);  v.im += dpp_z<0xB1>(v.im);
  v.re += dpp_z<0x4E>(v.re);  v.im += dpp_z<0x4E>(v.im);
  v.re += dpp_z<0x141>(v.re); v.im += dpp_z<0x141>(v.im);
  v.re += dpp_z<0x140>(v.re); v.im += dpp_z<0x140>(v.im);
  v.re += dpp_z<0x142>(v.re); v.im += dpp_z<0x142>(v.im);
  return {readlane_d(v.re, 31), readlane_d(v.im, 31)};
}

template <int CTRL>
__device__ inline dd dpp_dd(dd v) {
  return {dpp_z<CTRL>(v.hi), dpp_z<CTRL>(v.lo)};
}

// Double-double sum over the 64 lanes (dd_add at each level, the order of
// wsum).
__device__ inline dd wsum_dd(dd v) {
  v = dd_add(v, dpp_dd<0xB1>(v));
  v = dd_add(v, dpp_dd<0x4E>(v));
  v = dd_add(v, dpp_dd<0x141>(v));
  v = dd_add(v, dpp_dd<0x140>(v));
  v = dd_add(v, dpp_dd<0x142>(v));
  v = dd_add(v, dpp_dd<0x143>(v));
  return {readlane_d(v.hi, 63), readlane_d(v.lo, 63)};
}

// (e / n, e % n) without an integer division (float estimate, corrected).
__device__ inline void split_index(int e, int n, float rn, int& i, int& j) {
  i = (int)((float)e * rn);
  j = e - i * n;
  if (j >= n) { ++i; j -= n; }
  else if (j < 0) { --i; j += n; }
}

// Lanes of a wave over an m-column (or m-row) operation with a reduction
// along the other index: lane l serves column c = l mod m and the index
// range [j0, j1) of group l / m (g groups; lanes of group >= g are idle), so
// up to four lanes share a column's loop.  Partial results are combined in
// group order, so the sums do not depend on timing.
struct lane_split {
  int c, grp, g, j0, j1;
};

__device__ inline lane_split split_lanes(int m) {
  const int l = threadIdx.x;
  lane_split r;
  r.g = m <= 16 ? 4 : (m <= 21 ? 3 : (m <= 32 ? 2 : 1));
  r.grp = (int)((float)l / (float)m);      // exact: l < 64, m <= 64
  r.c = l - r.grp * m;
  const int span = (m + r.g - 1) / r.g;
  r.j0 = r.grp * span;
  r.j1 = r.grp < r.g ? min(m, r.j0 + span) : r.j0;
  return r;
}

// Sum of the g partial values part[grp * m + l] for lane l < m.
__device__ inline c64 combine_parts(const c64* part, const lane_split& sp, int m) {
  const int l = threadIdx.x;
  c64 v = {0.0, 0.0};
  if (l < m)
    for (int gr = 0; gr < sp.g; ++gr) v = v + part[gr * m + l];
  return v;
}

// ---------------------------------------------------------------- 1. tridiagonal
// Householder reduction of s.A (destroyed); T in s.a, s.b.  The trailing
// block's product p = A' v and its rank-2 update run on split lanes (up to
// four lanes per column), with the partial products combined through LDS.
__device__ inline void small_tridiag(small_ws& s, int n) {
  const int l = threadIdx.x;
  c64* __restrict__ A = s.A;
  c64* __restrict__ V = s.w;
  c64* __restrict__ W = s.u;
  c64* __restrict__ part = (c64*)s.part;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    const int o = k + 1;
    const lane_split sp = split_lanes(m);
    c64 xl = {0.0, 0.0};
    if (l < m) xl = conj(A[k * n + o + l]);     // A[o+l][k]
    const double x0r = readlane_d(xl.re, 0), x0i = readlane_d(xl.im, 0);
    const double ax0sq = x0r * x0r + x0i * x0i;
    const double r0 = rsq_nr(ax0sq > 0.0 ? ax0sq : 1.0);   // 1 / |x_0|, overlapping the sum below
    const double tail = wsum(l >= 1 ? norm2(xl) : 0.0);
    if (!(tail > 0.0)) {                        // column already reduced: reflector k = I
      if (l == 0) s.e[k] = {x0r, x0i};
      if (l < m) A[(size_t)(o + l) * n + k] = {0.0, 0.0};
      __syncthreads();
      continue;
    }
    const double s2 = ax0sq + tail;
    const double nx = s2 * rsq_nr(s2);
    const double ax0 = ax0sq > 0.0 ? ax0sq * r0 : 0.0;
    const c64 ph = ax0sq > 0.0 ? c64{x0r * r0, x0i * r0} : c64{1.0, 0.0};
    const c64 alpha = {-ph.re * nx, -ph.im * nx};
    const double sc = rsq_nr(nx * (nx + ax0));  // sqrt(2) / ||x - alpha e_0||
    c64 vl = {0.0, 0.0};
    if (l < m) {
      const c64 ul = (l == 0) ? c64{xl.re - alpha.re, xl.im - alpha.im} : xl;
      vl = {ul.re * sc, ul.im * sc};
      V[l] = vl;
      A[(size_t)(o + l) * n + k] = vl;          // reflector k, kept for the back-transformation
    }
    __syncthreads();
    // p = A' v (A' trailing m x m block; A'[c][j] = conj(A'[j][c]) read by column)
    {
      c64 p0 = {0.0, 0.0}, p1 = {0.0, 0.0};
      const c64* col = A + (size_t)o * n + o + sp.c;
      int j = sp.j0;
      for (; j + 4 <= sp.j1; j += 4) {
        const c64 a0 = col[(size_t)j * n], a1 = col[(size_t)(j + 1) * n];
        const c64 a2 = col[(size_t)(j + 2) * n], a3 = col[(size_t)(j + 3) * n];
        const c64 v0 = V[j], v1 = V[j + 1], v2 = V[j + 2], v3 = V[j + 3];
        p0 = p0 + cmulc(a0, v0) + cmulc(a2, v2);
        p1 = p1 + cmulc(a1, v1) + cmulc(a3, v3);
      }
      for (; j < sp.j1; ++j) p0 = p0 + cmulc(col[(size_t)j * n], V[j]);
      if (sp.grp < sp.g) part[l] = p0 + p1;
    }
    __syncthreads();
    const c64 pl = combine_parts(part, sp, m);
    const double K = 0.5 * wsum(l < m ? (vl.re * pl.re + vl.im * pl.im) : 0.0);  // Re(v^H p) / 2
    const c64 wl = {pl.re - K * vl.re, pl.im - K * vl.im};
    if (l < m) W[l] = wl;
    __syncthreads();
    // A' -= v w^H + w v^H   (lane (c, group) rewrites its rows of column c)
    if (sp.grp < sp.g) {
      const c64 cw = conj(W[sp.c]), cv = conj(V[sp.c]);
      c64* col = A + (size_t)o * n + o + sp.c;
      int j = sp.j0;
      for (; j + 4 <= sp.j1; j += 4) {
        c64 a0 = col[(size_t)j * n], a1 = col[(size_t)(j + 1) * n];
        c64 a2 = col[(size_t)(j + 2) * n], a3 = col[(size_t)(j + 3) * n];
        const c64 v0 = V[j], v1 = V[j + 1], v2 = V[j + 2], v3 = V[j + 3];
        const c64 w0 = W[j], w1 = W[j + 1], w2 = W[j + 2], w3 = W[j + 3];
        a0 = a0 - v0 * cw - w0 * cv;
        a1 = a1 - v1 * cw - w1 * cv;
        a2 = a2 - v2 * cw - w2 * cv;
        a3 = a3 - v3 * cw - w3 * cv;
        col[(size_t)j * n] = a0;
        col[(size_t)(j + 1) * n] = a1;
        col[(size_t)(j + 2) * n] = a2;
        col[(size_t)(j + 3) * n] = a3;
      }
      for (; j < sp.j1; ++j) {
        const c64 a0 = col[(size_t)j * n];
        col[(size_t)j * n] = a0 - V[j] * cw - W[j] * cv;
      }
    }
    if (l == 0) s.e[k] = alpha;
    __syncthreads();
  }
  if (l < n) s.a[l] = A[l * n + l].re;
  if (l == 0 && n >= 2) s.e[n - 2] = A[(n - 1) * n + n - 2];
  __syncthreads();
  if (l < n - 1) s.b[l] = sqrt(norm2(s.e[l]));
  if (l == n - 1) s.b[l] = 0.0;
  __syncthreads();
}

// ---------------------------------------------------------------- 2. bisection
// Number of eigenvalues of T below t (Sturm count).
__device__ inline int sturm_count(const double* a, const double* b, int n, double t, double pivmin) {
  double q = a[0] - t;
  int c = q < 0.0;
  for (int k = 1; k < n; ++k) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = a[k] - t - b[k - 1] * b[k - 1] * rcp_nr(q);
    c += q < 0.0;
  }
  return c;
}

// Bracket of the (target-1)-th smallest eigenvalue of T (target 1 or 2),
// 64 probes per round.  Returns ||T|| (Gershgorin bound) in *tn.
__device__ inline void small_bisect(const small_ws& s, int n, int target, double* lo_out, double* hi_out,
                                    double* tn_out) {
  const int l = threadIdx.x;
  double glo = 1.7976931348623157e308, ghi = -1.7976931348623157e308, bmax = 0.0;
  if (l < n) {
    const double bl = l > 0 ? s.b[l - 1] : 0.0, br = s.b[l];
    glo = s.a[l] - bl - br;
    ghi = s.a[l] + bl + br;
    bmax = br;
  }
  glo = wmin(glo);
  ghi = wmax(ghi);
  bmax = wmax(bmax);
  const double tn = fmax(fabs(glo), fabs(ghi));
  const double pivmin = fmax(bmax * bmax, 1e-280) * 1e-290 + 1e-300;
  double lo = glo - 2.2e-16 * tn - 1e-300, hi = ghi + 2.2e-16 * tn + 1e-300;
  for (int it = 0; it < SMALL_BISECT_ROUNDS; ++it) {
    const double h = (hi - lo) * (1.0 / 65.0);
    const bool hit = sturm_count(s.a, s.b, n, lo + h * (double)(l + 1), pivmin) >= target;
    const unsigned long long mask = __ballot(hit);
    const int js = mask ? __builtin_ctzll(mask) : 64;   // first probe above the eigenvalue
    const double nlo = js == 0 ? lo : lo + h * (double)js;
    const double nhi = js == 64 ? hi : lo + h * (double)(js + 1);
    lo = nlo;
    hi = nhi;
  }
  *lo_out = lo;
  *hi_out = hi;
  *tn_out = tn;
}

// ---------------------------------------------------------------- extreme-eigenvalue ratio
// Workspace of a reduction without eigenvectors (the matrix, three complex
// vectors, the real tridiagonal and the split-lane partial sums).
__host__ __device__ inline size_t small_probe_lds_bytes(int n) {
  return (size_t)n * n * sizeof(c64) + 3 * (size_t)n * sizeof(c64) + 2 * (size_t)n * sizeof(double) +
         (size_t)64 * sizeof(c64);
}

__device__ inline small_ws small_probe_carve(char* base, int n) {
  small_ws s = {};
  char* p = base;
  s.A = (c64*)p; p += (size_t)n * n * sizeof(c64);
  s.e = (c64*)p; p += n * sizeof(c64);
  s.w = (c64*)p; p += n * sizeof(c64);
  s.u = (c64*)p; p += n * sizeof(c64);
  s.a = (double*)p; p += n * sizeof(double);
  s.b = (double*)p; p += n * sizeof(double);
  s.part = (dd*)p;   // 64 complex partial sums (the reduction's split lanes)
  return s;
}

// lambda_min / lambda_max of the Hermitian positive semidefinite matrix in
// s.A (n x n, destroyed): Householder tridiagonalisation, then Sturm
// multisection brackets of the smallest and the largest eigenvalue (their
// midpoints; the smallest clamped at 0).  Wave-uniform; 0 for a zero matrix.
__device__ inline double small_extreme_ratio(small_ws& s, int n) {
  small_tridiag(s, n);
  double lo0, hi0, lo1, hi1, tn;
  small_bisect(s, n, 1, &lo0, &hi0, &tn);
  small_bisect(s, n, n, &lo1, &hi1, &tn);
  const double lmin = fmax(0.5 * (lo0 + hi0), 0.0), lmax = 0.5 * (lo1 + hi1);
  return lmax > 0.0 ? lmin / lmax : 0.0;
}

// Every eigenvalue of T on a log scale: lane l < n returns its (l+1)-th
// smallest eigenvalue, bisected in log10 over [1e-15 ||T||, ||T||] to
// SPECTRUM_ITERS steps (values below the range return its bottom).  Used for
// the learned form's features, which floor at 1e-14 of the largest
// eigenvalue.
constexpr int SPECTRUM_ITERS = 28;

__device__ inline double small_spectrum(const small_ws& s, int n) {
  const int l = threadIdx.x;
  double ghi = -1.7976931348623157e308, bmax = 0.0;
  if (l < n) {
    const double bl = l > 0 ? s.b[l - 1] : 0.0, br = s.b[l];
    ghi = s.a[l] + bl + br;
    bmax = br;
  }
  ghi = wmax(ghi);
  bmax = wmax(bmax);
  const double pivmin = fmax(bmax * bmax, 1e-280) * 1e-290 + 1e-300;
  const double top = log10(fmax(ghi, 1e-300));
  double lo = top - 15.0, hi = top;
  if (l < n) {
    for (int it = 0; it < SPECTRUM_ITERS; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (sturm_count(s.a, s.b, n, exp10(mid), pivmin) >= l + 1) hi = mid;
      else lo = mid;
    }
  }
  return exp10(0.5 * (lo + hi));
}

// ---------------------------------------------------------------- Gauss-Jordan inverse
// (used by the learned form's assembly)
// s.A <- s.A^{-1} for a Hermitian positive definite matrix (Gauss-Jordan, no
// pivoting; row and column k are staged in s.u / s.w before the update).
__device__ inline void small_gj_inverse(small_ws& s, int n) {
  const int l = threadIdx.x;
  const float rn = 1.0f / (float)n;
  const int nn = n * n;
  c64* __restrict__ A = s.A;
  c64* __restrict__ col = s.w;
  c64* __restrict__ row = s.u;
  for (int k = 0; k < n; ++k) {
    if (l < n) {
      col[l] = A[l * n + k];
      row[l] = A[k * n + l];
    }
    __syncthreads();
    const double ip = rcp_nr(row[k].re);
    for (int e0 = 0; e0 < nn; e0 += 8 * SMALL_NT) {
      c64 av[8], cv[8], rv[8];
      int ii[8], jj[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int e = e0 + l + t * SMALL_NT;
        split_index(e, n, rn, ii[t], jj[t]);
        if (e < nn) {
          av[t] = A[e];
          cv[t] = col[ii[t]];
          rv[t] = row[jj[t]];
        }
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int e = e0 + l + t * SMALL_NT;
        if (e < nn) {
          c64 v;
          if (ii[t] == k && jj[t] == k) v = {ip, 0.0};
          else if (ii[t] == k) v = ip * rv[t];
          else if (jj[t] == k) v = -ip * cv[t];
          else v = av[t] - ip * (cv[t] * rv[t]);
          A[e] = v;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- 3. tridiagonal solves
// The recurrences below are serial in k.  Every lane runs them in step on the
// same values read from LDS (broadcast reads, eight entries per batch, so the
// reads overlap the arithmetic of the previous batch); lane 0 stores the
// results.

// LDL^T factors of T - sigma I into s.w[k] = {1/d_k, l_k = b_k / d_k}
// (d_0 = a_0 - sigma, d_{k+1} = a_{k+1} - sigma - b_k l_k).  Pivots at or
// below pivmin (reachable only through rounding, since T - sigma I is
// positive definite) are raised to it.
__device__ inline void tri_factor(small_ws& s, int n, double sigma, double pivmin) {
  const int l = threadIdx.x;
  double d = s.a[0] - sigma;
  for (int k0 = 0; k0 < n; k0 += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + t;
      av[t] = k + 1 < n ? s.a[k + 1] : 0.0;
      bv[t] = k < n ? s.b[k] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + t;
      if (k < n) {
        if (!(d > pivmin)) d = pivmin;
        const double id = rcp_nr(d);
        const double lk = bv[t] * id;
        if (l == 0) s.w[k] = {id, lk};
        d = av[t] - sigma - bv[t] * lk;
      }
    }
  }
  __syncthreads();
}

// X = (T - sigma I)^{-1} (real symmetric) from the factors in s.w: lane j
// solves for column j (forward L w = e_j, w'_k = w_k / d_k, backward
// L^T z = w'), the factors being broadcast reads.
__device__ inline void build_x(small_ws& s, int n) {
  const int l = threadIdx.x;
  double* X = s.X;
  __syncthreads();
  if (l < n) {
    double w = 0.0, lprev = 0.0;
    for (int k0 = 0; k0 < n; k0 += 8) {
      c64 fv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) fv[t] = k0 + t < n ? s.w[k0 + t] : c64{0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = k0 + t;
        if (k < n) {
          w = (k == l ? 1.0 : 0.0) - lprev * w;
          lprev = fv[t].im;
          X[(size_t)k * n + l] = w * fv[t].re;
        }
      }
    }
    double z = 0.0;
    for (int k1 = n - 1; k1 >= 0; k1 -= 8) {
      double wv[8], lv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = k1 - t;
        wv[t] = k >= 0 ? X[(size_t)k * n + l] : 0.0;
        lv[t] = (k >= 0 && k + 1 < n) ? s.w[k].im : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = k1 - t;
        if (k >= 0) {
          z = wv[t] - lv[t] * z;
          X[(size_t)k * n + l] = z;
        }
      }
    }
  }
  __syncthreads();
}

// out_c = sum_{j < n} f(c, j) for lane c < n, on split lanes (f reads LDS).
template <class F>
__device__ inline c64 split_sum(small_ws& s, int n, F f) {
  const int l = threadIdx.x;
  const lane_split sp = split_lanes(n);
  c64 a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
  int j = sp.j0;
  for (; j + 4 <= sp.j1; j += 4) {
    const c64 f0 = f(sp.c, j), f1 = f(sp.c, j + 1), f2 = f(sp.c, j + 2), f3 = f(sp.c, j + 3);
    a0 = a0 + f0 + f2;
    a1 = a1 + f1 + f3;
  }
  for (; j < sp.j1; ++j) a0 = a0 + f(sp.c, j);
  c64* part = (c64*)s.part;
  if (sp.grp < sp.g) part[l] = a0 + a1;
  __syncthreads();
  const c64 r = combine_parts(part, sp, n);
  __syncthreads();
  return r;
}

// X r for lane-distributed r (staged in s.u); lane c returns entry c (zero
// for c >= n).  X is symmetric, so entry c is read along column c.
__device__ inline c64 x_mul(small_ws& s, int n, c64 r) {
  const int l = threadIdx.x;
  c64* b = s.u;
  __syncthreads();
  if (l < n) b[l] = r;
  __syncthreads();
  const double* X = s.X;
  return split_sum(s, n, [&](int c, int k) __attribute__((always_inline)) {
    const double x = X[(size_t)k * n + c];
    const c64 bk = b[k];
    return c64{x * bk.re, x * bk.im};
  });
}

// Diagonal unitary D with D^H T_c D = T (T_c the complex tridiagonal with
// subdiagonal e_k, T its real form with b_k = |e_k|): ph_0 = 1,
// ph_{k+1} = ph_k e_k / |e_k|, i.e. lane k receives the product of the unit
// factors of e_0 .. e_{k-1} (an inclusive product scan over the lanes by DPP
// row shifts and row broadcasts; zero for lanes >= n).
template <int CTRL, int ROWMASK>
__device__ inline c64 scan_mul_step(c64 x) {
  const c64 y = {dpp_d<CTRL, ROWMASK>(x.re, 1.0), dpp_d<CTRL, ROWMASK>(x.im, 0.0)};   // absent lanes give 1
  return x * y;
}

__device__ inline c64 tri_phases(const small_ws& s, int n) {
  const int l = threadIdx.x;
  c64 t = {1.0, 0.0};
  if (l >= 1 && l < n) {
    const double ae = s.b[l - 1];
    if (ae > 0.0) {
      const c64 e = s.e[l - 1];
      const double ir = rcp_nr(ae);
      t = {e.re * ir, e.im * ir};
    }
  }
  t = scan_mul_step<0x111, 0xf>(t);   // row_shr:1
  t = scan_mul_step<0x112, 0xf>(t);   // row_shr:2
  t = scan_mul_step<0x114, 0xf>(t);   // row_shr:4
  t = scan_mul_step<0x118, 0xf>(t);   // row_shr:8
  t = scan_mul_step<0x142, 0xa>(t);   // row_bcast:15 into rows 1, 3
  t = scan_mul_step<0x143, 0xc>(t);   // row_bcast:31 into rows 2, 3
  return l < n ? t : c64{0.0, 0.0};
}

// Q y (adjoint false) or Q^H y (adjoint true) for Q = H_0 H_1 ... H_{n-3},
// H_k = I - v_k v_k^H, v_k kept in column k below the diagonal of s.A (zero
// for an identity step).  Lane l holds y_l (zero for l >= n); each reflector
// costs one wave sum.  Reflector entries are read eight at a time from
// clamped (always valid) addresses and zeroed where they lie outside v_k.
template <bool HALF>
__device__ inline __attribute__((always_inline)) c64 q_apply_w(const small_ws& s, int n, c64 y, bool adjoint) {
  const int l = threadIdx.x;
  const int nr = n - 2;
  const int ll = min(l, n - 1);
  const c64* __restrict__ row = s.A + (size_t)ll * n;
  for (int t0 = 0; t0 < nr; t0 += 8) {
    c64 vv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = min(t0 + u, nr - 1);
      const int k = adjoint ? t : nr - 1 - t;
      vv[u] = row[k];
      if (!(l > k && l < n)) vv[u] = {0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (t0 + u < nr) {
        const c64 d = HALF ? wsum_c32(cmulc(vv[u], y)) : wsum_c(cmulc(vv[u], y));
        y = y - vv[u] * d;
      }
    }
  }
  return y;
}

__device__ inline __attribute__((always_inline)) c64 q_apply(const small_ws& s, int n, c64 y, bool adjoint) {
  return n <= 32 ? q_apply_w<true>(s, n, y, adjoint) : q_apply_w<false>(s, n, y, adjoint);
}

// ---------------------------------------------------------------- the solver
// acc.get(i, j) gives G in double-double; G's rounded value must already be
// in s.A (destroyed).  Leaves the unit eigenvector in s.x (lane l also keeps
// entry l) and *steps the number of refinement steps.  With want_diag it
// returns mu = x^H G x (dd) of that vector and *lam1 receives the second
// smallest eigenvalue; without, both are NaN (the product G x of the final
// vector serves only mu, so it is skipped).  max_refine bounds the Newton
// steps: 0 leaves the inverse-iteration vector.
template <class Acc>
__device__ inline dd small_eig(small_ws& s, const Acc& acc, int n, bool want_diag, double* lam1, int* steps,
                               int max_refine = SMALL_REFINE_MAX) {
  const int l = threadIdx.x;
  if (n == 1) {
    if (l == 0) s.x[0] = {1.0, 0.0};
    __syncthreads();
    *lam1 = __builtin_nan("");
    *steps = 0;
    return want_diag ? acc.get(0, 0).re : dd{__builtin_nan(""), 0.0};
  }
  small_tridiag(s, n);
  double lo0, hi0, tn;
  small_bisect(s, n, 1, &lo0, &hi0, &tn);
  if (want_diag) {
    double lo1, hi1, tn1;
    small_bisect(s, n, 2, &lo1, &hi1, &tn1);
    *lam1 = 0.5 * (lo1 + hi1);
  } else {
    *lam1 = __builtin_nan("");
  }
  const double sigma = lo0 - 16.0 * n * 2.2e-16 * tn;
  const double pivmin = 1e-300 + 2.2e-16 * 2.2e-16 * tn;
  tri_factor(s, n, sigma, pivmin);
  const c64 ph = tri_phases(s, n);
  build_x(s, n);
  // inverse iteration on T from a fixed, generic start vector, then x = W y
  c64 y = l < n ? c64{1.0 + 0.6180339887 * (double)((l * 7) % 11), 0.0} : c64{0.0, 0.0};
  for (int it = 0; it < SMALL_INVIT; ++it) {
    y = x_mul(s, n, y);
    const double nr = sqrt(wsum(norm2(y)));
    y = {y.re / nr, y.im / nr};
  }
  c64 xl = q_apply(s, n, y * ph, false);
  {
    const double nr = sqrt(wsum(l < n ? norm2(xl) : 0.0));
    xl = l < n ? c64{xl.re / nr, xl.im / nr} : c64{0.0, 0.0};
  }
  if (l < n) s.x[l] = xl;
  __syncthreads();
  if (max_refine == 0 && !want_diag) {
    *steps = 0;
    return dd{__builtin_nan(""), 0.0};
  }
  // Newton refinement against the double-double matrix.  The product G x is
  // split over ng lane groups (lane l: row l mod n, columns of group l / n),
  // whose partial sums are added in group order.
  const int ng = n <= 16 ? 4 : (n <= 21 ? 3 : (n <= 32 ? 2 : 1));
  const int row = l % n, grp = l / n;
  const int jspan = (n + ng - 1) / ng;
  const int j0 = grp * jspan, j1 = min(n, j0 + jspan);
  dd mu = {0.0, 0.0};
  double dprev = 0.0;
  int it = 0;
  bool done = false;
  for (;; ++it) {
    if (grp < ng) {
      dot2 ar, ai;
      ar.init();
      ai.init();
      for (int j = j0; j < j1; ++j) {
        const cdd g = acc.get(row, j);
        const c64 xj = s.x[j];
        ar.add_prod(g.re.hi, xj.re); ar.add(g.re.lo * xj.re);
        ar.add_prod(-g.im.hi, xj.im); ar.add(-g.im.lo * xj.im);
        ai.add_prod(g.re.hi, xj.im); ai.add(g.re.lo * xj.im);
        ai.add_prod(g.im.hi, xj.re); ai.add(g.im.lo * xj.re);
      }
      s.part[2 * l] = ar.result();
      s.part[2 * l + 1] = ai.result();
    }
    __syncthreads();
    dd yre = {0.0, 0.0}, yim = {0.0, 0.0};
    if (l < n) {
      yre = s.part[2 * l];
      yim = s.part[2 * l + 1];
      for (int g = 1; g < ng; ++g) {
        yre = dd_add(yre, s.part[2 * (g * n + l)]);
        yim = dd_add(yim, s.part[2 * (g * n + l) + 1]);
      }
    }
    __syncthreads();
    dot2 t;
    t.init();
    t.add_prod(xl.re, yre.hi); t.add(xl.re * yre.lo);
    t.add_prod(xl.im, yim.hi); t.add(xl.im * yim.lo);
    mu = wsum_dd(t.result());
    if (done || it == max_refine) break;
    c64 r = {0.0, 0.0};
    if (l < n) {
      dot2 qr, qi;
      qr.init(); qi.init();
      qr.add_dd(yre); qr.add_prod(-mu.hi, xl.re); qr.add(-mu.lo * xl.re);
      qi.add_dd(yim); qi.add_prod(-mu.hi, xl.im); qi.add(-mu.lo * xl.im);
      r = {dd_val(qr.result()), dd_val(qi.result())};
    }
    // correction c = W (T - sigma I)^{-1} W^H r
    const c64 t1 = cmulc(ph, q_apply(s, n, r, true));
    const c64 t2 = x_mul(s, n, t1);
    const c64 cl = q_apply(s, n, t2 * ph, false);
    const c64 xn = l < n ? xl - cl : c64{0.0, 0.0};
    const double nrm = sqrt(wsum(norm2(xn)));
    // the change of direction: with c = alpha x + c_perp, x - c turns by
    // |c_perp| / |1 - alpha| (the part along x, which M amplifies from the
    // rounding of r, only rescales x)
    const c64 al = wsum_c(l < n ? cmulc(xl, cl) : c64{0.0, 0.0});
    const c64 cp = l < n ? cl - xl * al : c64{0.0, 0.0};
    const double dn = sqrt(wsum(norm2(cp))) / sqrt((1.0 - al.re) * (1.0 - al.re) + al.im * al.im);
    xl = {xn.re / nrm, xn.im / nrm};
    __syncthreads();
    if (l < n) s.x[l] = xl;
    __syncthreads();
    // converged when the change of direction, or the next one predicted from
    // the linear rate dn / dprev of the last two, is below 4e-15
    done = !(dn > 4e-15) || (dprev > 0.0 && dn * dn <= 4e-15 * dprev);
    dprev = dn;
    if (done && !want_diag) {
      ++it;
      mu = {__builtin_nan(""), 0.0};
      break;
    }
  }
  *steps = it;
  return mu;
}

}  // namespace cbp
