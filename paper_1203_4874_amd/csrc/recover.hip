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
  __device__ cdd get(int i, int j) const {
    if (i < k2) {
      if (j < k2) {
        const int l = i - j;
        return l >= 0 ? rho[l] : cdd_conj(rho[-l]);
      }
      const int q = j - k2;
      return cdd_neg(rho[k2 + k1 + (i - q) + (k1 - 1)]);
    }
    const int p = i - k2;
    if (j >= k2) {
      const int l = p - (j - k2);
      return l >= 0 ? rho[k2 + l] : cdd_conj(rho[k2 - l]);
    }
    return cdd_conj(cdd_neg(rho[k2 + k1 + (j - p) + (k1 - 1)]));
  }
};

// Scale system H from its diagonal blocks (Da, Db) and coupling C.
struct scale_acc {
  const dd* Da;
  const dd* Db;
  const cdd* C;
  int S;
  __device__ cdd get(int r, int c) const {
    const dd z = {0.0, 0.0};
    if (r < S && c < S) return r == c ? cdd{Da[r], z} : cdd{z, z};
    if (r >= S && c >= S) return r == c ? cdd{Db[r - S], z} : cdd{z, z};
    if (r < S) return C[r * S + (c - S)];
    return cdd_conj(C[c * S + (r - S)]);
  }
};

__device__ inline void unit_twiddles(c64* tw, int S) {
  for (int t = threadIdx.x; t < S; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)S, &s, &c);
    tw[t] = {c, s};
  }
}

__device__ inline bool finite_c(c64 v) { return isfinite(v.re) && isfinite(v.im); }

// Correlations rho for every (pass, sample, lag), summed over channels.
// grid (2N-1, S, 2), one wave each; Dot2 accumulation per lane, then a
// fixed-order double-double wave reduction.
__global__ __launch_bounds__(64) void k_gram(const c64* ex, const c64* ey, int Wmax, int Hmax, int W1, int W2,
                                             int H1, int H2, int S, int k1, int k2, int nch, cdd* corr) {
  const int li = blockIdx.x, j = blockIdx.y, pass = blockIdx.z;
  const int N = k1 + k2, NL = 2 * N - 1;
  int fa, fb, l;
  if (li < k2) { fa = 0; fb = 0; l = li; }
  else if (li < k2 + k1) { fa = 1; fb = 1; l = li - k2; }
  else { fa = 0; fb = 1; l = li - (k1 + k2) - (k1 - 1); }
  const int la = pass == 0 ? (fa ? W2 : W1) : (fa ? H2 : H1);
  const int lb = pass == 0 ? (fb ? W2 : W1) : (fb ? H2 : H1);
  const int stride = pass == 0 ? Wmax : Hmax;
  const c64* base = pass == 0 ? ex : ey;
  const int t0 = max(0, -l), t1 = min(la, lb - l);
  dot2 sre, sim;
  sre.init();
  sim.init();
  for (int ch = 0; ch < nch; ++ch) {
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
  if (threadIdx.x == 0) corr[((size_t)pass * S + j) * NL + li] = cdd{re, im};
}

// Smallest eigenvector of every per-sample Gram.  grid (S, 2), one wave each.
__global__ __launch_bounds__(SMALL_NT) void k_sample(const cdd* corr, int S, int k1, int k2, c64* xout,
                                                     double* lam0, cbp_diag* diag) {
  extern __shared__ __attribute__((aligned(16))) char sm_sample[];
  const int N = k1 + k2, NL = 2 * N - 1;
  const int j = blockIdx.x, pass = blockIdx.y;
  const int l = threadIdx.x;
  cdd* rho = (cdd*)sm_sample;
  small_ws w = small_carve(sm_sample + (((size_t)NL * sizeof(cdd) + 15) & ~(size_t)15), N);
  for (int t = l; t < NL; t += SMALL_NT) rho[t] = corr[((size_t)pass * S + j) * NL + t];
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
  const dd mu = small_eig(w, G, N, diag != nullptr, &lam1, &steps);
  const size_t base = ((size_t)pass * S + j) * N;
  const c64 xi = l < N ? w.x[l] : c64{0.0, 0.0};
  if (l < N) {
    xout[base + l] = xi;
    if (diag) {
      diag->sample_vec[pass][j][l][0] = xi.re;
      diag->sample_vec[pass][j][l][1] = xi.im;
    }
  }
  const bool bad = wmax(l < N && !finite_c(xi) ? 1.0 : 0.0) > 0.0;
  if (l == 0) {
    const double l0 = dd_val(mu);
    lam0[pass * S + j] = l0;
    if (diag) {
      diag->sample_lambda0[pass][j] = l0;
      diag->sample_lambda1[pass][j] = lam1;
      diag->sample_scale[pass][j] = gmax;
      atomicMax(&diag->refine_sample, steps);
      if (!(lam1 - l0 > 1e-13 * gmax)) atomicOr(&diag->flags, CBP_DIAG_SAMPLE_WEAK);  // NaN-safe: flags NaN too
      if (bad || !isfinite(l0)) atomicOr(&diag->flags, CBP_DIAG_NONFINITE);
    }
  }
}

// Scale fix, assembly, inverse DFT and normalisation.  One wave.
__global__ __launch_bounds__(SMALL_NT) void k_finalize(const c64* xvec, int S, int k1, int k2, c64* pq, cdd* cbuf,
                                                       double* K1, double* K2, cbp_diag* diag) {
  extern __shared__ __attribute__((aligned(16))) char sm_fin[];
  const int N = k1 + k2, n2 = 2 * S, SS = S * S;
  const int tid = threadIdx.x;
  c64* tw = (c64*)sm_fin;                        // S
  dd* Da = (dd*)(tw + CBP_MAX_S);                // S
  dd* Db = Da + CBP_MAX_S;                       // S
  small_ws w = small_carve((char*)(Db + CBP_MAX_S), n2);
  // after the scale solve, its matrix region (4 S^2 entries) holds the
  // averaged spectra / inverse DFTs (2 S^2) and the half-transformed ones (2 S^2)
  c64* kbuf = w.A;
  c64* tbuf = w.A + 2 * SS;
  unit_twiddles(tw, S);
  __syncthreads();
  // cofactors evaluated on the other axis: pq = [P1, P2, Q1, Q2], each [i][j]
  for (int e = tid; e < 4 * SS; e += SMALL_NT) {
    const int which = e / SS, ij = e - which * SS;
    const int i = ij / S, jj = ij - i * S;
    const c64* xs;
    int len, f;
    if (which == 0) { xs = xvec + ((size_t)jj) * N + k2; len = k1; f = i; }          // P1: v of pass X sample jj
    else if (which == 1) { xs = xvec + ((size_t)jj) * N; len = k2; f = i; }          // P2: u of pass X sample jj
    else if (which == 2) { xs = xvec + ((size_t)S + i) * N + k2; len = k1; f = jj; } // Q1: v of pass Y sample i
    else { xs = xvec + ((size_t)S + i) * N; len = k2; f = jj; }                      // Q2: u of pass Y sample i
    c64 acc = {0.0, 0.0};
    int t = 0;
    for (int x = 0; x < len; ++x) {
      acc = acc + xs[x] * tw[t];
      t += f;
      if (t >= S) t -= S;
    }
    pq[e] = acc;
  }
  __threadfence_block();
  __syncthreads();
  // H blocks in double-double
  for (int e = tid; e < SS; e += SMALL_NT) {
    const int jj = e / S, i = e - jj * S;
    dot2 re, im;
    re.init();
    im.init();
    for (int c = 0; c < 2; ++c) {
      const c64 P = pq[(size_t)c * SS + i * S + jj], Q = pq[(size_t)(2 + c) * SS + i * S + jj];
      re.add_prod(-P.re, Q.re); re.add_prod(-P.im, Q.im);
      im.add_prod(-P.re, Q.im); im.add_prod(P.im, Q.re);
    }
    cbuf[e] = cdd{re.result(), im.result()};
  }
  for (int t = tid; t < n2; t += SMALL_NT) {
    dot2 d;
    d.init();
    if (t < S) {
      for (int c = 0; c < 2; ++c)
        for (int i = 0; i < S; ++i) {
          const c64 P = pq[(size_t)c * SS + i * S + t];
          d.add_prod(P.re, P.re); d.add_prod(P.im, P.im);
        }
      Da[t] = d.result();
    } else {
      const int i = t - S;
      for (int c = 0; c < 2; ++c)
        for (int jj = 0; jj < S; ++jj) {
          const c64 Q = pq[(size_t)(2 + c) * SS + i * S + jj];
          d.add_prod(Q.re, Q.re); d.add_prod(Q.im, Q.im);
        }
      Db[i] = d.result();
    }
  }
  __threadfence_block();
  __syncthreads();
  const scale_acc H{Da, Db, cbuf, S};
  for (int e = tid; e < n2 * n2; e += SMALL_NT) {
    const int r = e / n2, c = e - r * n2;
    const cdd h = H.get(r, c);
    w.A[e] = {h.re.hi, h.im.hi};
  }
  const double hmax = wmax(tid < n2 ? dd_val(H.get(tid, tid).re) : 0.0);
  __syncthreads();
  double lam1;
  int steps;
  const dd mu = small_eig(w, H, n2, diag != nullptr, &lam1, &steps);
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
  for (int e = tid; e < 2 * SS; e += SMALL_NT) {
    const int c = e / SS, ij = e - c * SS;
    const int i = ij / S, jj = ij - i * S;
    const c64 P = pq[(size_t)c * SS + ij], Q = pq[(size_t)(2 + c) * SS + ij];
    const c64 v = w.x[jj] * P + w.x[S + i] * Q;
    Kh[e] = {0.5 * v.re, 0.5 * v.im};
    if (diag) {
      diag->khat[c][i][jj][0] = 0.5 * v.re;
      diag->khat[c][i][jj][1] = 0.5 * v.im;
    }
  }
  __syncthreads();
  // inverse DFT along x: Tm[c][j][x] = sum_i Kh[c][i][j] w_i^{-x}
  for (int e = tid; e < 2 * SS; e += SMALL_NT) {
    const int c = e / SS, jx = e - c * SS;
    const int jj = jx / S, x = jx - jj * S;
    c64 acc = {0.0, 0.0};
    int t = 0;
    for (int i = 0; i < S; ++i) {
      acc = acc + Kh[(size_t)c * SS + i * S + jj] * conj(tw[t]);
      t += x;
      if (t >= S) t -= S;
    }
    Tm[e] = acc;
  }
  __syncthreads();
  // inverse DFT along y: Kf[c][y][x] = sum_j w_j^{-y} Tm[c][j][x]   (into Kh)
  for (int e = tid; e < 2 * SS; e += SMALL_NT) {
    const int c = e / SS, yx = e - c * SS;
    const int y = yx / S, x = yx - y * S;
    c64 acc = {0.0, 0.0};
    int t = 0;
    for (int jj = 0; jj < S; ++jj) {
      acc = acc + Tm[(size_t)c * SS + jj * S + x] * conj(tw[t]);
      t += y;
      if (t >= S) t -= S;
    }
    Kh[e] = acc;
  }
  __syncthreads();
  for (int c = 0; c < 2; ++c) {
    const int k = c == 0 ? k1 : k2;
    double sr = 0.0, si = 0.0, ein = 0.0, eall = 0.0;
    for (int e = tid; e < SS; e += SMALL_NT) {
      const int y = e / S, x = e - y * S;
      const c64 v = Kh[(size_t)c * SS + e];
      const double p = norm2(v);
      eall += p;
      if (y < k && x < k) { sr += v.re; si += v.im; ein += p; }
    }
    sr = wsum(sr);
    si = wsum(si);
    ein = wsum(ein);
    eall = wsum(eall);
    const double s2 = sr * sr + si * si;
    double* K = c == 0 ? K1 : K2;
    double re2 = 0.0, im2 = 0.0;
    for (int e = tid; e < k * k; e += SMALL_NT) {
      const int y = e / k, x = e - y * k;
      const c64 v = Kh[(size_t)c * SS + y * S + x];
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
      diag->kernel_outside[c] = (eall - ein) / fmax(eall, 1e-300);
      if (!(s2 > 0.0) || !isfinite(s2)) atomicOr(&diag->flags, CBP_DIAG_KERNEL_ZERO);
      if (!isfinite(re2)) atomicOr(&diag->flags, CBP_DIAG_NONFINITE);
    }
  }
}

__global__ void k_diag_init(cbp_diag* diag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    diag->flags = 0;
    diag->refine_sample = 0;
    diag->refine_scale = 0;
  }
}

}  // namespace

size_t finalize_lds_bytes(int S) {
  return (size_t)CBP_MAX_S * sizeof(c64) + 2 * (size_t)CBP_MAX_S * sizeof(dd) + small_lds_bytes(2 * S);
}

size_t sample_lds_bytes(int N) {
  return ((((size_t)(2 * N - 1) * sizeof(cdd)) + 15) & ~(size_t)15) + small_lds_bytes(N);
}

hipError_t launch_recover(const frame_plan& fp, char* ws, double* K1, double* K2, void* diagp, hipStream_t st) {
  static bool attrs_set = false;
  if (!attrs_set) {
    hipFuncSetAttribute((const void*)k_sample, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipFuncSetAttribute((const void*)k_finalize, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attrs_set = true;
  }
  cbp_diag* diag = (cbp_diag*)diagp;
  const int S = fp.S, N = fp.N;
  const c64* ex = (const c64*)(ws + fp.off_ex);
  const c64* ey = (const c64*)(ws + fp.off_ey);
  cdd* corr = (cdd*)(ws + fp.off_corr);
  c64* xvec = (c64*)(ws + fp.off_xvec);
  double* lam0 = (double*)(ws + fp.off_lam0);
  if (diag) hipLaunchKernelGGL(k_diag_init, dim3(1), dim3(256), 0, st, diag);
  prof_begin(PH_GRAM, st);
  hipLaunchKernelGGL(k_gram, dim3(2 * N - 1, S, 2), dim3(64), 0, st, ex, ey, fp.Wmax, fp.Hmax, fp.W1, fp.W2, fp.H1,
                     fp.H2, S, fp.k1, fp.k2, fp.nch, corr);
  prof_end(PH_GRAM, st);
  prof_begin(PH_SAMPLE, st);
  hipLaunchKernelGGL(k_sample, dim3(S, 2), dim3(SMALL_NT), sample_lds_bytes(N), st, corr, S, fp.k1, fp.k2, xvec,
                     lam0, diag);
  prof_end(PH_SAMPLE, st);
  prof_begin(PH_FINALIZE, st);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(SMALL_NT), finalize_lds_bytes(S), st, xvec, S, fp.k1, fp.k2,
                     (c64*)(ws + fp.off_pq), (cdd*)(ws + fp.off_cbuf), K1, K2, diag);
  prof_end(PH_FINALIZE, st);
  return hipGetLastError();
}

}  // namespace cbp
