// Kernel recovery on the GPU: per-sample Gram matrices, their smallest
// eigenvectors (the 1-D cofactors), the two-order scale fix and the assembly
// of the kernels (Sec. 4 and Sec. 5).
//
// Per sample j of pass X (and i of pass Y) the 1-D cofactors solve
//   b1(w_j, .) (x) u = b2(w_j, .) (x) v,   u: k2 taps, v: k1 taps,
// since b1 k2 = l k1 k2 = b2 k1 (eq. 4).  With A = [C_k2(e1) | -C_k1(e2)]
// (C_k(e) the full-convolution matrix of e), the Gram G = A^H A is block
// Toeplitz:
//   G11[p][q] = rho11(p - q),  G22[p][q] = rho22(p - q),  G12[p][q] = -rho12(p - q),
//   rho_ab(l) = sum_t conj(a[t]) b[t + l],
// so only 2(k1+k2)-1 correlations are formed, each accumulated in
// double-double (Dot2).  The null vector x = (u, v) is the eigenvector of the
// smallest eigenvalue of G (eigsmall.h).
//
// Scale fix (Sec. 4: combine the two evaluation orders by least squares;
// Sec. 5: 2t unknowns over t x t equations): with the cofactors evaluated on
// the other axis,
//   P_c[i][j] = sum_x v_j^{(c)}[x] w_i^x   (pass X slice j),
//   Q_c[i][j] = sum_y v_i'^{(c)}[y] w_j^y  (pass Y slice i),
// the scales z = (a, b) minimise sum_{c,i,j} |a_j P_c[i][j] - b_i Q_c[i][j]|^2
// with ||z|| = 1: the smallest eigenvector of
//   H = [[diag(sum |P|^2), -C], [-C^H, diag(sum |Q|^2)]],  C[j][i] = sum_c conj(P_c[i][j]) Q_c[i][j].
// Assembly (Sec. 5, abstract): Khat_c = (a_j P_c + b_i Q_c) / 2, inverse
// S x S DFT, crop to the k_c x k_c support, divide by the complex sum over
// the support and keep the real part.
#include "eigsmall.h"
#include "internal.h"

namespace cbp {

namespace {

// G of one sample from its correlations rho (stored: rho11[0..k2),
// rho22[0..k1), rho12[-(k1-1)..k2-1]).
struct gram_acc {
  const cdd* rho;
  int k1, k2;
  // Row i varies across lanes, column j is uniform: one index and two sign
  // choices, no divergent branches.
  __device__ cdd get(int i, int j) const {
    const bool ia = i < k2, ja = j < k2;
    const int lag = i - j;
    const int cross = k2 + k1 + (k1 - 1);
    int idx;
    bool cj, ng;
    if (ia == ja) {                      // G11 or G22: rho_aa(i - j), conj for negative lags
      idx = (ia ? 0 : k2) + (lag < 0 ? -lag : lag);
      cj = lag < 0;
      ng = false;
    } else {                             // G12 = -rho12(p - q), G21 = G12^H
      idx = ia ? cross + i - (j - k2) : cross + j - (i - k2);
      cj = !ia;
      ng = true;
    }
    cdd v = rho[idx];
    if (cj) v.im = dd_neg(v.im);
    if (ng) v = cdd_neg(v);
    return v;
  }
};

// Scale system H from its diagonal blocks (Da, Db) and coupling C.
struct scale_acc {
  const dd* Da;
  const dd* Db;
  const cdd* C;
  int S;
  __device__ __attribute__((always_inline)) cdd get(int r, int c) const {
    const dd z = {0.0, 0.0};
    if (r < S && c < S) return r == c ? cdd{Da[r], z} : cdd{z, z};
    if (r >= S && c >= S) return r == c ? cdd{Db[r - S], z} : cdd{z, z};
    if (r < S) return C[r * S + (c - S)];
    return cdd_conj(C[c * S + (r - S)]);
  }
};

__device__ inline bool finite_c(c64 v) { return isfinite(v.re) && isfinite(v.im); }

// Both kernels to zero (each lane clears the entries it wrote): a pair whose
// estimate is non-finite or sums to zero is returned as zeros, so that the
// Fourier division that follows writes a zero latent instead of spreading
// the non-finite values.
__device__ inline void zero_kernels(double* K1, int k1, double* K2, int k2) {
  for (int e = threadIdx.x; e < k1 * k1; e += SMALL_NT) K1[e] = 0.0;
  for (int e = threadIdx.x; e < k2 * k2; e += SMALL_NT) K2[e] = 0.0;
}

// Correlations rho for every (pass, sample, lag), summed over channels.
// Items: (lag, sample, pass), one wave each; Dot2 accumulation per lane,
// then a fixed-order double-double wave reduction.
__global__ __launch_bounds__(64) void k_gram(batch_ref br) {
  for_items<Q_GRAM>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int k1 = d.k1, k2 = d.k2, S = d.S;
    const int N = k1 + k2, NL = 2 * N - 1;
    const int li = item % NL, rest = item / NL;
    const int j = rest % S, pass = rest / S;
    int fa, fb, l;
    if (li < k2) { fa = 0; fb = 0; l = li; }
    else if (li < k2 + k1) { fa = 1; fb = 1; l = li - k2; }
    else { fa = 0; fb = 1; l = li - (k1 + k2) - (k1 - 1); }
    // fields into locals first: a select between fields would select between
    // their addresses and keep the descriptor copy out of registers
    const int W1 = d.W1, W2 = d.W2, H1 = d.H1, H2 = d.H2, Wmax = d.Wmax, Hmax = d.Hmax;
    const c64* ex = d.ex;
    const c64* ey = d.ey;
    const int la = pass == 0 ? (fa ? W2 : W1) : (fa ? H2 : H1);
    const int lb = pass == 0 ? (fb ? W2 : W1) : (fb ? H2 : H1);
    const int stride = pass == 0 ? Wmax : Hmax;
    const c64* base = pass == 0 ? ex : ey;
    const int t0 = max(0, -l), t1 = min(la, lb - l);
    dot2 sre, sim;
    sre.init();
    sim.init();
    for (int ch = 0; ch < d.nch; ++ch) {
      const c64* a = base + ((size_t)(ch * 2 + fa) * S + j) * stride;
      const c64* b = base + ((size_t)(ch * 2 + fb) * S + j) * stride;
      int t = t0 + (int)threadIdx.x;
      for (; t + 64 < t1; t += 128) {
        const c64 a0 = a[t], b0 = b[t + l], a1 = a[t + 64], b1 = b[t + 64 + l];
        sre.add_prod(a0.re, b0.re); sre.add_prod(a0.im, b0.im);
        sim.add_prod(a0.re, b0.im); sim.add_prod(-a0.im, b0.re);
        sre.add_prod(a1.re, b1.re); sre.add_prod(a1.im, b1.im);
        sim.add_prod(a1.re, b1.im); sim.add_prod(-a1.im, b1.re);
      }
      if (t < t1) {
        const c64 a0 = a[t], b0 = b[t + l];
        sre.add_prod(a0.re, b0.re); sre.add_prod(a0.im, b0.im);
        sim.add_prod(a0.re, b0.im); sim.add_prod(-a0.im, b0.re);
      }
    }
    const dd re = wsum_dd(sre.result());
    const dd im = wsum_dd(sim.result());
    if (threadIdx.x == 0) d.corr[((size_t)pass * S + j) * NL + li] = cdd{re, im};
  });
}

// Smallest eigenvector of every per-sample Gram.  Items: (sample, pass),
// one wave each.
__global__ __launch_bounds__(SMALL_NT) void k_sample(batch_ref br) {
  extern __shared__ __attribute__((aligned(16))) char sm_sample[];
  __shared__ c64 twq[CBP_MAX_S];
  for_items<Q_SAMPLE>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int k1 = d.k1, k2 = d.k2, S = d.S;
    const int N = k1 + k2, NL = 2 * N - 1;
    const int j = item % S, pass = item / S;
    const int l = threadIdx.x;
    cbp_diag* diag = d.diag;
    cdd* rho = (cdd*)sm_sample;
    small_ws w = small_carve(sm_sample + (((size_t)NL * sizeof(cdd) + 15) & ~(size_t)15), N, false);
    for (int t = l; t < NL; t += SMALL_NT) rho[t] = d.corr[((size_t)pass * S + j) * NL + t];
    __syncthreads();
    const gram_acc G{rho, k1, k2};
    for (int e = l; e < N * N; e += SMALL_NT) {
      const int i = e / N, c = e - i * N;
      const cdd g = G.get(i, c);
      w.A[e] = {g.re.hi, g.im.hi};
    }
    const double gmax = wmax(l < N ? dd_val(G.get(l, l).re) : 0.0);
    __syncthreads();
    double lam1;
    int steps;
    const dd mu = small_eig(w, G, N, diag != nullptr, &lam1, &steps, solve_refine_max(d.variant));
    const size_t base = ((size_t)pass * S + j) * N;
    const c64 xi = l < N ? w.x[l] : c64{0.0, 0.0};
    if (l < N) {
      d.xvec[base + l] = xi;
      if (diag) {
        diag->sample_vec[pass][j][l][0] = xi.re;
        diag->sample_vec[pass][j][l][1] = xi.im;
      }
    }
    // the scale fix's cofactors evaluated on the other axis, this sample's
    // share: pass X sample j gives P_c[.][j], pass Y sample i gives Q_c[i][.]
    // (c = 0: the v part, k1 taps; c = 1: the u part, k2 taps)
    if (l < S) {
      double sn, cs;
      sincospi(-2.0 * (double)l / (double)S, &sn, &cs);
      twq[l] = {cs, sn};
    }
    __syncthreads();
    if (l < 2 * S) {
      const int c = l < S ? 0 : 1, f = l - c * S;
      const c64* xs = c == 0 ? w.x + k2 : w.x;
      const int len = c == 0 ? k1 : k2;
      c64 acc = {0.0, 0.0};
      int t = 0;
      for (int x = 0; x < len; ++x) {
        acc = acc + xs[x] * twq[t];
        t += f;
        if (t >= S) t -= S;
      }
      const size_t SS = (size_t)S * S;
      if (pass == 0) d.pq[c * SS + (size_t)f * S + j] = acc;        // P_c[i = f][j]
      else d.pq[(2 + c) * SS + (size_t)j * S + f] = acc;             // Q_c[i = j][jj = f]
    }
    const bool bad = wmax(l < N && !finite_c(xi) ? 1.0 : 0.0) > 0.0;
    if (d.feat) {
      // learned form (and diagnostics): features of this sample's spectrum
      // (the tridiagonal T of the solve is still in w.a / w.b):
      //   f_i = log10(max(lambda_i, 1e-14 lambda_max) / lambda_max) / 10, i < N; +1 after
      const double lam = small_spectrum(w, N);
      const double lmax = readlane_d(lam, N - 1);
      if (l < 32) {
        const float f = l < N ? (float)(log10(fmax(lam, 1e-14 * lmax) / lmax) * 0.1) : 1.0f;
        d.feat[((size_t)pass * S + j) * 32 + l] = f;
        if (diag) diag->sample_features[pass][j][l] = f;
      }
    }
    if (l == 0) {
      const double l0 = dd_val(mu);
      if (diag) {
        diag->sample_lambda0[pass][j] = l0;
        diag->sample_lambda1[pass][j] = lam1;
        diag->sample_scale[pass][j] = gmax;
        atomicMax(&diag->refine_sample, steps);
        if (!(lam1 - l0 > 1e-13 * gmax)) atomicOr(&diag->flags, CBP_DIAG_SAMPLE_WEAK);  // NaN-safe: flags NaN too
        if (bad || !isfinite(l0)) atomicOr(&diag->flags, CBP_DIAG_NONFINITE);
      }
    }
  });
}

// Scale fix, assembly, inverse DFT and normalisation.  One wave.
// Learned form (wts != NULL): wts[j] = wX_j (pass-X sample j), wts[S + i] =
// wY_i, wts[2S] = tau.  The scale system's rows are weighted by
// sqrt(wX_j wY_i); the spectra are averaged with weights wX_j, wY_i; each
// kernel Z = K^T (k x k, [x][y]) solves (Ax + tau I) Z (By + tau I) = C with
//   Ax = Fx^H D_u Fx, By = Fy^T D_v conj(Fy), C = Fx^H D_u Khat D_v conj(Fy),
// u = wY, v = wX, F[i][x] = w_i^x (the separable weighted fit with per-axis
// Tikhonov terms), then is divided by its complex sum (real part kept).
__device__ inline __attribute__((always_inline)) bool learned_assembly(const c64* tw, int S, int k, const double* wts, c64* Kh, c64* tb, c64* xt,
                                        double* K, cbp_diag* diag, int c);

// LDS of the plain finalize: twiddles, the two diagonal blocks, the solver.
// lean: the scale solve keeps no caller half (see finalize_frame).
__host__ __device__ inline size_t fin_base_bytes(int S, bool lean = false) {
  return (size_t)CBP_MAX_S * sizeof(c64) + 2 * (size_t)CBP_MAX_S * sizeof(dd) + small_lds_bytes(2 * S, !lean);
}

// Kernels from the per-sample scales: both kernels' normalisation (divide by
// the complex sum over the support, keep the real part) and diagnostics;
// F1 / F2 hold each kernel's S x S (row stride S) inverse transform.  Returns
// true when a kernel is non-finite or sums to zero (wave-uniform).
__device__ inline __attribute__((always_inline)) bool normalise_kernels(const c64* F1, const c64* F2, int S, int k1,
                                                                         int k2, double* K1, double* K2,
                                                                         cbp_diag* diag) {
  const int tid = threadIdx.x, SS = S * S;
  const float rS = 1.0f / (float)S;
  bool bad = false;
  for (int c = 0; c < 2; ++c) {
    const int k = c == 0 ? k1 : k2;
    const c64* F = c == 0 ? F1 : F2;
    const float rk = 1.0f / (float)k;
    double sr = 0.0, si = 0.0, ein = 0.0, eall = 0.0;
    for (int e = tid; e < SS; e += SMALL_NT) {
      int y, x;
      split_index(e, S, rS, y, x);
      const c64 v = F[e];
      const double p = norm2(v);
      eall += p;
      if (y < k && x < k) { sr += v.re; si += v.im; ein += p; }
    }
    {   // pairs of sums share a reduction (each component in wsum's order)
      const c64 a = wsum_c(c64{sr, si}), b = wsum_c(c64{ein, eall});
      sr = a.re;
      si = a.im;
      ein = b.re;
      eall = b.im;
    }
    const double s2 = sr * sr + si * si;
    double* K = c == 0 ? K1 : K2;
    double re2 = 0.0, im2 = 0.0;
    for (int e = tid; e < k * k; e += SMALL_NT) {
      int y, x;
      split_index(e, k, rk, y, x);
      const c64 v = F[y * S + x];
      const double kr = (v.re * sr + v.im * si) / s2;
      const double ki = (v.im * sr - v.re * si) / s2;
      K[e] = kr;
      re2 += kr * kr;
      im2 += ki * ki;
    }
    {
      const c64 q = wsum_c(c64{re2, im2});
      re2 = q.re;
      im2 = q.im;
    }
    if (tid == 0 && diag) {
      diag->kernel_imag[c] = sqrt(im2) / fmax(sqrt(re2), 1e-300);
      diag->kernel_outside[c] = (eall - ein) / fmax(eall, 1e-300);
      if (!(s2 > 0.0) || !isfinite(s2)) atomicOr(&diag->flags, CBP_DIAG_KERNEL_ZERO);
      if (!isfinite(re2)) atomicOr(&diag->flags, CBP_DIAG_NONFINITE);
    }
    bad = bad || !(s2 > 0.0) || !isfinite(s2) || !isfinite(re2);   // wave-uniform
  }
  return bad;
}

// Scale system of the one-axis fix (S x S, double-double entries in LDS).
struct cdd_mat_acc {
  const cdd* H;
  int n;
  __device__ cdd get(int r, int c) const { return H[r * n + c]; }
};

// The one-axis scale fix (the paper's scales from one evaluation order,
// fixed by the kernels' finite support).  With the pass-X null vectors X_j
// (u: kernel 2's slice, k2 taps; v: kernel 1's slice, k1 taps) and a_j the
// scale of sample j, the inverse DFT over j of a_j X^c_j[x] must vanish at
// rows k_c <= y < S.  The Gram of those equations is
//   H[j][j'] = sum_c (sum_{x < k_c} conj(X^c_j[x]) X^c_j'[x]) g_c(j - j'),
//   g_c(t) = sum_{y = k_c}^{S-1} w^{t y},  w = exp(-2 pi i / S),
// and a is its smallest eigenvector; K_c[y][x] = (1/S) sum_j a_j X^c_j[x] w_j^{-y}.
__device__ inline __attribute__((always_inline)) void one_axis_frame(const c64* xvec, int S, int k1, int k2,
                                                                      double* K1, double* K2, cbp_diag* diag,
                                                                      char* sm_fin, int variant) {
  const int N = k1 + k2, SS = S * S, tid = threadIdx.x;
  const float rS = 1.0f / (float)S;
  c64* tw = (c64*)sm_fin;                                   // S
  c64* X = tw + CBP_MAX_S;                                  // [S][N]
  char* after = (char*)(X + (((size_t)S * N + 1) & ~(size_t)1));
  small_ws w = small_carve(after, S);
  cdd* Hm = (cdd*)(after + small_lds_bytes(S));             // [S][S]
  unit_twiddles(tw, S);
  for (int e = tid; e < S * N; e += SMALL_NT) X[e] = xvec[e];   // pass X: [j][l]
  __syncthreads();
  for (int e = tid; e < SS; e += SMALL_NT) {
    int j, jp;
    split_index(e, S, rS, j, jp);
    int t = j - jp;
    if (t < 0) t += S;
    dot2 re, im;
    re.init();
    im.init();
    for (int c = 0; c < 2; ++c) {
      const int k = c == 0 ? k1 : k2, o = c == 0 ? k2 : 0;
      dot2 sre, sim;
      sre.init();
      sim.init();
      for (int x = 0; x < k; ++x) {
        const c64 a = X[j * N + o + x], b = X[jp * N + o + x];
        sre.add_prod(a.re, b.re); sre.add_prod(a.im, b.im);
        sim.add_prod(a.re, b.im); sim.add_prod(-a.im, b.re);
      }
      c64 g = {0.0, 0.0};
      int ty = (t * k) % S;
      for (int y = k; y < S; ++y) {
        g = g + tw[ty];
        ty += t;
        if (ty >= S) ty -= S;
      }
      const dd sr = sre.result(), si = sim.result();
      re.add_prod(sr.hi, g.re); re.add_prod(sr.lo, g.re); re.add_prod(-si.hi, g.im); re.add_prod(-si.lo, g.im);
      im.add_prod(sr.hi, g.im); im.add_prod(sr.lo, g.im); im.add_prod(si.hi, g.re); im.add_prod(si.lo, g.re);
    }
    Hm[e] = cdd{re.result(), im.result()};
  }
  __syncthreads();
  for (int e = tid; e < SS; e += SMALL_NT) w.A[e] = {Hm[e].re.hi, Hm[e].im.hi};
  const cdd_mat_acc H{Hm, S};
  const double hmax = wmax(tid < S ? dd_val(Hm[tid * S + tid].re) : 0.0);
  __syncthreads();
  double lam1;
  int steps;
  const dd mu = small_eig(w, H, S, diag != nullptr, &lam1, &steps, solve_refine_max(variant));
  if (tid == 0 && diag) {
    diag->k1 = k1; diag->k2 = k2; diag->S = S; diag->n = N;
    diag->scale_lambda0 = dd_val(mu);
    diag->scale_lambda1 = lam1;
    diag->scale_scale = hmax;
    diag->refine_scale = steps;
    if (!(lam1 - dd_val(mu) > 1e-13 * hmax)) atomicOr(&diag->flags, CBP_DIAG_SCALE_WEAK);
  }
  if (diag)
    for (int t = tid; t < S; t += SMALL_NT) {
      diag->scale_vec[t][0] = w.x[t].re;
      diag->scale_vec[t][1] = w.x[t].im;
    }
  __syncthreads();
  // F[c][y][x] = (1/S) sum_j a_j X^c_j[x] w_j^{-y}  (into the solver's matrix region, 2 S^2 entries)
  c64* F = w.A;    // kernel 1: the solver's matrix region (S^2 entries, free after the solve)
  c64* F2 = w.W;   // kernel 2: its W region (S (S + 1) entries)
  const double rs = 1.0 / (double)S;
  for (int e = tid; e < 2 * SS; e += SMALL_NT) {
    const int c = e >= SS, yx = e - c * SS;
    int y, x;
    split_index(yx, S, rS, y, x);
    const int k = c == 0 ? k1 : k2, o = c == 0 ? k2 : 0;
    c64 acc = {0.0, 0.0};
    if (x < k) {
      int t = 0;
      for (int j = 0; j < S; ++j) {
        acc = acc + (w.x[j] * X[j * N + o + x]) * conj(tw[t]);
        t += y;
        if (t >= S) t -= S;
      }
    }
    (c == 0 ? F : F2)[yx] = {acc.re * rs, acc.im * rs};
  }
  __syncthreads();
  if (normalise_kernels(F, F2, S, k1, k2, K1, K2, diag)) zero_kernels(K1, k1, K2, k2);
}

__device__ inline __attribute__((always_inline)) void finalize_frame(const c64* xvec, int S, int k1, int k2, c64* pq, double* K1,
                                      double* K2, cbp_diag* diag, char* sm_fin, const double* wts, int variant) {
  if (variant & VAR_ONE_AXIS) {
    one_axis_frame(xvec, S, k1, k2, K1, K2, diag, sm_fin, variant);
    return;
  }
  // kernel 1's equations only (the k1-only scale least squares) or both kernels'
  const int nc = (variant & VAR_SCALE_K1) ? 1 : 2;
  const int N = k1 + k2, n2 = 2 * S, SS = S * S;
  const int tid = threadIdx.x;
  const float rS = 1.0f / (float)S, rSS = 1.0f / (float)SS, rn2 = 1.0f / (float)n2;
  c64* tw = (c64*)sm_fin;                        // S
  dd* Da = (dd*)(tw + CBP_MAX_S);                // S
  dd* Db = Da + CBP_MAX_S;                       // S
  // The coupling block (below) is read through H by the Newton refinement
  // and by the diagnostics' Rayleigh quotient after the solver has built X;
  // a solve with neither reads it only before (A and hmax come from it), so
  // it may share X's region (lean: no caller half, 9 KB less LDS at S = 17,
  // which lets the workgroup fit on a CU beside the FFT passes' workgroups).
  const bool lean = solve_refine_max(variant) == 0 && diag == nullptr;
  small_ws w = small_carve((char*)(Db + CBP_MAX_S), n2, !lean);
  // after the scale solve, its matrix region (4 S^2 entries) holds the
  // averaged spectra / inverse DFTs (2 S^2) and the half-transformed ones (2 S^2)
  c64* kbuf = w.A;
  c64* tbuf = w.A + 2 * SS;
  unit_twiddles(tw, S);
  // the cofactors evaluated on the other axis, pq = [P1, P2, Q1, Q2] (each
  // [i][j], written by the sample solves), staged in the solver's matrix
  // region (4 S^2 entries, filled with H's rounding once they are read); the
  // coupling block C (S^2 double-double entries) goes to the W region, which
  // the solver leaves free (or, lean, which it fills with X only after C's
  // last read), so every read of H is an LDS read
  c64* pql = w.A;
  cdd* cmat = (cdd*)w.W;
  for (int e0 = 0; e0 < 4 * SS; e0 += 8 * SMALL_NT) {   // eight loads in flight per lane
    c64 v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = e0 + tid + t * SMALL_NT;
      v[t] = e < 4 * SS ? pq[e] : c64{0.0, 0.0};
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = e0 + tid + t * SMALL_NT;
      if (e < 4 * SS) pql[e] = v[t];
    }
  }
  __syncthreads();
  // H blocks in double-double
  for (int e = tid; e < SS; e += SMALL_NT) {
    int jj, i;
    split_index(e, S, rS, jj, i);
    dot2 re, im;
    re.init();
    im.init();
    const double W = wts ? wts[jj] * wts[S + i] : 1.0;
    for (int c = 0; c < nc; ++c) {
      c64 P = pql[(size_t)c * SS + i * S + jj];
      const c64 Q = pql[(size_t)(2 + c) * SS + i * S + jj];
      if (wts) P = {W * P.re, W * P.im};
      re.add_prod(-P.re, Q.re); re.add_prod(-P.im, Q.im);
      im.add_prod(-P.re, Q.im); im.add_prod(P.im, Q.re);
    }
    cmat[e] = cdd{re.result(), im.result()};
  }
  // diagonal blocks: Da[t] = sum over (c, i) of w |P_c[i][t]|^2, Db[t] =
  // sum over (c, j) of w |Q_c[t][j]|^2, in that order, with the entries
  // read eight at a time (clamped indices; the extra reads are not summed)
  for (int t = tid; t < n2; t += SMALL_NT) {
    const bool isa = t < S;
    const int tt = isa ? t : t - S;
    dot2 d;
    d.init();
    const int nq = nc * S;
    for (int q0 = 0; q0 < nq; q0 += 8) {
      c64 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = min(q0 + u, nq - 1);
        const int c = q >= S, r = q - c * S;
        v[u] = pql[isa ? (size_t)c * SS + r * S + tt : (size_t)(2 + c) * SS + tt * S + r];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u;
        if (q < nq) {
          const int r = q >= S ? q - S : q;
          if (wts) {
            const double W = isa ? wts[tt] * wts[S + r] : wts[r] * wts[S + tt];
            d.add_prod(W * v[u].re, v[u].re);
            d.add_prod(W * v[u].im, v[u].im);
          } else {
            d.add_prod(v[u].re, v[u].re);
            d.add_prod(v[u].im, v[u].im);
          }
        }
      }
    }
    if (isa) Da[tt] = d.result();
    else Db[tt] = d.result();
  }
  __threadfence_block();
  __syncthreads();
  const scale_acc H{Da, Db, cmat, S};
  for (int e = tid; e < n2 * n2; e += SMALL_NT) {
    int r, c;
    split_index(e, n2, rn2, r, c);
    const cdd h = H.get(r, c);
    w.A[e] = {h.re.hi, h.im.hi};
  }
  const double hmax = wmax(tid < n2 ? dd_val(H.get(tid, tid).re) : 0.0);
  __syncthreads();
  double lam1;
  int steps;
  const dd mu = small_eig(w, H, n2, diag != nullptr, &lam1, &steps, solve_refine_max(variant));
  if (tid == 0 && diag) {
    diag->k1 = k1; diag->k2 = k2; diag->S = S; diag->n = N;
    diag->scale_lambda0 = dd_val(mu);
    diag->scale_lambda1 = lam1;
    diag->scale_scale = hmax;
    diag->refine_scale = steps;
    if (!(lam1 - dd_val(mu) > 1e-13 * hmax)) atomicOr(&diag->flags, CBP_DIAG_SCALE_WEAK);
  }
  if (diag)
    for (int t = tid; t < n2; t += SMALL_NT) {
      diag->scale_vec[t][0] = w.x[t].re;
      diag->scale_vec[t][1] = w.x[t].im;
    }
  // averaged spectra Kh[c][i][j]
  c64* Kh = kbuf;
  c64* Tm = tbuf;
  for (int e0 = 0; e0 < 2 * SS; e0 += 4 * SMALL_NT) {
    c64 Pv[4], Qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {   // eight loads in flight per lane (indices clamped in range)
      const int e = min(e0 + tid + u * SMALL_NT, 2 * SS - 1);
      int c, ij;
      split_index(e, SS, rSS, c, ij);
      Pv[u] = pq[(size_t)c * SS + ij];
      Qv[u] = pq[(size_t)(2 + c) * SS + ij];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + tid + u * SMALL_NT;
      if (e >= 2 * SS) break;
      int c, ij;
      split_index(e, SS, rSS, c, ij);
      int i, jj;
      split_index(ij, S, rS, i, jj);
      const c64 P = Pv[u], Q = Qv[u];
      c64 kv;
      if (wts) {
        const double wx = wts[jj], wy = wts[S + i], r = 1.0 / (wx + wy);
        const c64 a = w.x[jj] * P, b = w.x[S + i] * Q;
        kv = {(wx * a.re + wy * b.re) * r, (wx * a.im + wy * b.im) * r};
      } else {
        const c64 v = w.x[jj] * P + w.x[S + i] * Q;
        kv = {0.5 * v.re, 0.5 * v.im};
      }
      Kh[e] = kv;
      if (diag) {
        diag->khat[c][i][jj][0] = kv.re;
        diag->khat[c][i][jj][1] = kv.im;
      }
    }
  }
  __syncthreads();
  if (wts) {
    if (diag)
      for (int t = tid; t <= n2; t += SMALL_NT) diag->sample_weights[t] = wts[t];
    c64* xt = w.W;   // S^2 + 2 CBP_MAX_S entries from the solver's W onwards (free after the solve)
    const bool bad1 = learned_assembly(tw, S, k1, wts, Kh, tbuf, xt, K1, diag, 0);
    const bool bad2 = learned_assembly(tw, S, k2, wts, Kh + SS, tbuf, xt, K2, diag, 1);
    if (bad1 || bad2) zero_kernels(K1, k1, K2, k2);
    return;
  }
  // inverse DFT along x: Tm[c][j][x] = sum_i Kh[c][i][j] w_i^{-x}, two
  // outputs per lane at a time (independent chains, each summed in i order)
  for (int e = tid; e < 2 * SS; e += 2 * SMALL_NT) {
    const int f = min(e + SMALL_NT, 2 * SS - 1);
    int c, jx, jj, x, c2, jx2, jj2, x2;
    split_index(e, SS, rSS, c, jx);
    split_index(jx, S, rS, jj, x);
    split_index(f, SS, rSS, c2, jx2);
    split_index(jx2, S, rS, jj2, x2);
    c64 acc = {0.0, 0.0}, acc2 = {0.0, 0.0};
    int t = 0, t2 = 0;
#pragma unroll 4
    for (int i = 0; i < S; ++i) {
      acc = acc + Kh[(size_t)c * SS + i * S + jj] * conj(tw[t]);
      acc2 = acc2 + Kh[(size_t)c2 * SS + i * S + jj2] * conj(tw[t2]);
      t += x;
      if (t >= S) t -= S;
      t2 += x2;
      if (t2 >= S) t2 -= S;
    }
    Tm[e] = acc;
    if (e + SMALL_NT < 2 * SS) Tm[f] = acc2;
  }
  __syncthreads();
  // inverse DFT along y: Kf[c][y][x] = sum_j w_j^{-y} Tm[c][j][x]   (into Kh),
  // two outputs per lane at a time as above
  for (int e = tid; e < 2 * SS; e += 2 * SMALL_NT) {
    const int f = min(e + SMALL_NT, 2 * SS - 1);
    int c, yx, y, x, c2, yx2, y2, x2;
    split_index(e, SS, rSS, c, yx);
    split_index(yx, S, rS, y, x);
    split_index(f, SS, rSS, c2, yx2);
    split_index(yx2, S, rS, y2, x2);
    c64 acc = {0.0, 0.0}, acc2 = {0.0, 0.0};
    int t = 0, t2 = 0;
#pragma unroll 4
    for (int jj = 0; jj < S; ++jj) {
      acc = acc + Tm[(size_t)c * SS + jj * S + x] * conj(tw[t]);
      acc2 = acc2 + Tm[(size_t)c2 * SS + jj * S + x2] * conj(tw[t2]);
      t += y;
      if (t >= S) t -= S;
      t2 += y2;
      if (t2 >= S) t2 -= S;
    }
    Kh[e] = acc;
    if (e + SMALL_NT < 2 * SS) Kh[f] = acc2;
  }
  __syncthreads();
  if (normalise_kernels(Kh, Kh + SS, S, k1, k2, K1, K2, diag)) zero_kernels(K1, k1, K2, k2);
}

// Returns true when the kernel is non-finite or sums to zero (wave-uniform).
__device__ inline __attribute__((always_inline)) bool learned_assembly(const c64* tw, int S, int k, const double* wts, c64* Kh, c64* tb, c64* xt,
                                        double* K, cbp_diag* diag, int c) {
  const int tid = threadIdx.x, kk = k * k;
  const float rS = 1.0f / (float)S, rk = 1.0f / (float)k;
  const double tau = wts[2 * S];
  c64* Ax = tb;             // k x k
  c64* By = tb + kk;        // k x k
  c64* T1 = xt;             // k x S, later Z1 (k x k)
  c64* Cm = Kh;             // k x k, over Khat once T1 is formed
  // F[i][x] = w_i^x = tw[(i x) mod S];  u_i = wY_i,  v_j = wX_j
  for (int e = tid; e < kk; e += SMALL_NT) {
    int p, q;
    split_index(e, k, rk, p, q);
    c64 a = {0.0, 0.0}, b = {0.0, 0.0};
    for (int i = 0; i < S; ++i) {
      const c64 fp = tw[(i * p) % S], fq = tw[(i * q) % S];
      const c64 g = cmulc(fp, fq);            // conj(F[i][p]) F[i][q]
      a = a + c64{wts[S + i] * g.re, wts[S + i] * g.im};
      const c64 h = cmulc(fq, fp);            // F[j][p] conj(F[j][q])
      b = b + c64{wts[i] * h.re, wts[i] * h.im};
    }
    if (p == q) { a.re += tau; b.re += tau; }
    Ax[e] = a;
    By[e] = b;
  }
  // T1[x][j] = sum_i conj(F[i][x]) u_i Khat[i][j]
  for (int e = tid; e < k * S; e += SMALL_NT) {
    int x, jj;
    split_index(e, S, rS, x, jj);
    c64 acc = {0.0, 0.0};
    for (int i = 0; i < S; ++i) {
      const c64 g = cmulc(tw[(i * x) % S], Kh[i * S + jj]);
      acc = acc + c64{wts[S + i] * g.re, wts[S + i] * g.im};
    }
    T1[e] = acc;
  }
  __syncthreads();
  // C[x][y] = sum_j T1[x][j] v_j conj(F[j][y])
  for (int e = tid; e < kk; e += SMALL_NT) {
    int x, y;
    split_index(e, k, rk, x, y);
    c64 acc = {0.0, 0.0};
    for (int jj = 0; jj < S; ++jj) {
      const c64 g = cmulc(tw[(jj * y) % S], T1[x * S + jj]);
      acc = acc + c64{wts[jj] * g.re, wts[jj] * g.im};
    }
    Cm[e] = acc;
  }
  __syncthreads();
  // (Ax + tau I)^{-1}, (By + tau I)^{-1} in place (Hermitian positive definite)
  small_ws g;
  g.w = xt + (size_t)S * S;
  g.u = g.w + CBP_MAX_S;
  g.A = Ax;
  small_gj_inverse(g, k);
  g.A = By;
  small_gj_inverse(g, k);
  // Z1 = Ax^{-1} C (into T1), Z = Z1 By^{-1} (into Cm)
  for (int e = tid; e < kk; e += SMALL_NT) {
    int x, y;
    split_index(e, k, rk, x, y);
    c64 acc = {0.0, 0.0};
    for (int t = 0; t < k; ++t) acc = acc + Ax[x * k + t] * Cm[t * k + y];
    T1[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < kk; e += SMALL_NT) {
    int x, y;
    split_index(e, k, rk, x, y);
    c64 acc = {0.0, 0.0};
    for (int t = 0; t < k; ++t) acc = acc + T1[x * k + t] * By[t * k + y];
    Cm[e] = acc;
  }
  __syncthreads();
  // K[y][x] = Z[x][y] / sum(Z), real part
  double sr = 0.0, si = 0.0;
  for (int e = tid; e < kk; e += SMALL_NT) { sr += Cm[e].re; si += Cm[e].im; }
  sr = wsum(sr);
  si = wsum(si);
  const double s2 = sr * sr + si * si;
  double re2 = 0.0, im2 = 0.0;
  for (int e = tid; e < kk; e += SMALL_NT) {
    int y, x;
    split_index(e, k, rk, y, x);
    const c64 v = Cm[x * k + y];
    const double kr = (v.re * sr + v.im * si) / s2;
    const double ki = (v.im * sr - v.re * si) / s2;
    K[e] = kr;
    re2 += kr * kr;
    im2 += ki * ki;
  }
  re2 = wsum(re2);
  im2 = wsum(im2);
  if (tid == 0 && diag) {
    diag->kernel_imag[c] = sqrt(im2) / fmax(sqrt(re2), 1e-300);
    diag->kernel_outside[c] = 0.0;
    if (!(s2 > 0.0) || !isfinite(s2)) atomicOr(&diag->flags, CBP_DIAG_KERNEL_ZERO);
    if (!isfinite(re2)) atomicOr(&diag->flags, CBP_DIAG_NONFINITE);
  }
  __syncthreads();
  return !(s2 > 0.0) || !isfinite(s2) || !isfinite(re2);
}

// Items: one per frame.  plain_only: the plain method's kernels into the
// learned form's fallback slots (d.Kalt), ignoring the network's weights.
__global__ __launch_bounds__(SMALL_NT) void k_finalize(batch_ref br, int plain_only) {
  extern __shared__ __attribute__((aligned(16))) char sm_fin[];
  for_items<Q_FINALIZE>(br, [&](const frame_desc& d, int) __attribute__((always_inline)) {
    double* K1 = plain_only ? d.Kalt : d.K1;
    double* K2 = plain_only ? d.Kalt + CBP_MAX_K * CBP_MAX_K : d.K2;
    finalize_frame(d.xvec, d.S, d.k1, d.k2, d.pq, K1, K2, plain_only ? nullptr : d.diag, sm_fin,
                   plain_only ? nullptr : d.wts, d.variant);
  });
}

// The learned form's judge: the plain method's objective
//   J(K1, K2) = sum over passes and samples of x^H G x / x^H x,
// with x = (K2 slice, K1 slice) of the kernels at that sample (the
// per-sample TLS residual the plain method minimises), for the plain
// kernels (d.Kalt) and the learned ones (d.K1, d.K2); the plain ones replace
// the learned ones when their J is smaller, or when the frame is noisy (the
// regime where the network does not gain).  Items: one per frame.
constexpr float LEARNED_NOISY_F0 = -1.0f;
__global__ __launch_bounds__(64) void k_judge(batch_ref br) {
  __shared__ c64 tw[CBP_MAX_S];
  __shared__ c64 xs[CBP_MAX_N];
  for_items<Q_FINALIZE>(br, [&](const frame_desc& d, int) __attribute__((always_inline)) {
    const int S = d.S, k1 = d.k1, k2 = d.k2, N = k1 + k2, NL = 2 * N - 1;
    const int l = threadIdx.x;
    unit_twiddles(tw, S);
    __syncthreads();
    double J[2];
    for (int set = 0; set < 2; ++set) {
      const double* A1 = set ? d.K1 : d.Kalt;
      const double* A2 = set ? d.K2 : d.Kalt + CBP_MAX_K * CBP_MAX_K;
      double acc = 0.0;
      for (int pass = 0; pass < 2; ++pass)
        for (int j = 0; j < S; ++j) {
          if (l < N) {
            const bool u = l < k2;
            const double* K = u ? A2 : A1;
            const int k = u ? k2 : k1, c = u ? l : l - k2;
            c64 sacc = {0.0, 0.0};
            int t = 0;
            for (int r = 0; r < k; ++r) {
              const double kv = pass == 0 ? K[r * k + c] : K[c * k + r];   // along y (pass X) or x (pass Y)
              sacc = sacc + c64{kv * tw[t].re, kv * tw[t].im};
              t += j;
              if (t >= S) t -= S;
            }
            xs[l] = sacc;
          }
          __syncthreads();
          const gram_acc G{d.corr + ((size_t)pass * S + j) * NL, k1, k2};
          double num = 0.0, nx = 0.0;
          if (l < N) {
            c64 y = {0.0, 0.0};
            for (int q = 0; q < N; ++q) {
              const cdd g = G.get(l, q);
              y = y + c64{dd_val(g.re), dd_val(g.im)} * xs[q];
            }
            const c64 xl = xs[l];
            num = xl.re * y.re + xl.im * y.im;   // Re(conj(x_l) y_l)
            nx = norm2(xl);
          }
          num = wsum(num);
          nx = wsum(nx);
          acc += num / nx;
          __syncthreads();
        }
      J[set] = acc;
    }
    // the network's weights are used only on frames without a noise floor:
    // when more than half of the 2S samples have lambda_0 / lambda_max above
    // 1e-10 (spectrum feature f_0 > -1) the plain kernels are kept
    const float f0 = l < 2 * S ? d.feat[(size_t)l * 32] : -2.0f;   // sample rows (pass, j) in order
    const bool noisy = wsum(f0 > LEARNED_NOISY_F0 ? 1.0 : 0.0) > (double)S;
    // NaN-safe: the learned kernels are kept only when their objective is a
    // number no larger than the plain one's
    const bool fallback = noisy || !(J[1] <= J[0]);
    if (fallback) {
      for (int e = l; e < k1 * k1; e += 64) d.K1[e] = d.Kalt[e];
      for (int e = l; e < k2 * k2; e += 64) d.K2[e] = d.Kalt[CBP_MAX_K * CBP_MAX_K + e];
    }
    if (l == 0 && d.diag) {
      d.diag->judge[0] = J[0];
      d.diag->judge[1] = J[1];
      if (fallback) atomicOr(&d.diag->flags, CBP_DIAG_FALLBACK);
    }
  });
}

// Dense per-sample Gram matrices from the correlations (the a2 output of
// cbp_sample_grams): out[pass][j][p][q] = G(p, q) rounded to FP64.
// Items: (sample, pass).
__global__ __launch_bounds__(64) void k_gram_expand(batch_ref br, c64* out) {
  for_items<Q_GRAMM>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int S = d.S, N = d.N, NL = 2 * N - 1;
    const gram_acc G{d.corr + (size_t)item * NL, d.k1, d.k2};
    c64* o = out + (size_t)item * N * N;
    for (int e = threadIdx.x; e < N * N; e += 64) {
      const cdd g = G.get(e / N, e % N);
      o[e] = {dd_val(g.re), dd_val(g.im)};
    }
    (void)S;
  });
}

// Clear the per-call diagnostic counters.  Items: one per frame.
__global__ void k_diag_init(batch_ref br) {
  for_items<Q_DIAG>(br, [&](const frame_desc& d, int) __attribute__((always_inline)) {
    if (threadIdx.x == 0 && d.diag) {
      d.diag->flags = 0;
      d.diag->refine_sample = 0;
      d.diag->refine_scale = 0;
    }
  });
}

}  // namespace

// LDS of the finalize: the plain part (the coupling block lives in the
// solver's W region) and, for the learned assembly, T1 / Z1 (S^2) and the
// inversion's two vectors, taken from the same W region (2S (2S + 1)
// entries, the last region of the solver's LDS) plus what they need beyond
// it.
size_t finalize_lds_bytes(int S, int learned, bool lean) {
  const size_t base = fin_base_bytes(S, lean);
  const size_t need = ((size_t)S * S + 2 * CBP_MAX_S) * sizeof(c64);
  const size_t have = lean ? (size_t)(2 * S) * (2 * S) * sizeof(double) : (size_t)(2 * S) * (2 * S + 1) * sizeof(c64);
  return learned && need > have ? base + (need - have) : base;
}

size_t sample_lds_bytes(int N) {
  return ((((size_t)(2 * N - 1) * sizeof(cdd)) + 15) & ~(size_t)15) + small_lds_bytes(N, false);
}

void set_recover_attrs() {
  hipFuncSetAttribute((const void*)k_sample, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  hipFuncSetAttribute((const void*)k_finalize, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t launch_diag_init(const batch_ref& br, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_init, dim3(grid), dim3(64), 0, st, br);
  return hipGetLastError();
}

hipError_t launch_gram_expand(const batch_ref& br, int grid, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_expand, dim3(grid), dim3(64), 0, st, br, (c64*)out);
  return hipGetLastError();
}

hipError_t launch_gram(const batch_ref& br, int grid, hipStream_t st) {
  prof_begin(PH_GRAM, st);
  hipLaunchKernelGGL(k_gram, dim3(grid), dim3(64), 0, st, br);
  prof_end(PH_GRAM, st);
  return hipGetLastError();
}

hipError_t launch_sample(const batch_ref& br, int grid, int maxN, hipStream_t st) {
  prof_begin(PH_SAMPLE, st);
  hipLaunchKernelGGL(k_sample, dim3(grid), dim3(SMALL_NT), sample_lds_bytes(maxN), st, br);
  prof_end(PH_SAMPLE, st);
  return hipGetLastError();
}

hipError_t launch_judge(const batch_ref& br, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_judge, dim3(grid), dim3(64), 0, st, br);
  return hipGetLastError();
}

hipError_t launch_finalize(const batch_ref& br, int grid, int maxS, int learned, int plain_only, bool lean,
                           hipStream_t st) {
  prof_begin(PH_FINALIZE, st);
  hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(SMALL_NT), finalize_lds_bytes(maxS, learned, lean), st, br,
                     plain_only);
  prof_end(PH_FINALIZE, st);
  return hipGetLastError();
}

}  // namespace cbp
