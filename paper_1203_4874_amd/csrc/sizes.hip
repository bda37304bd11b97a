// Blind kernel-size estimation (Sec. 4: the first stage finds the kernel
// degree from the singularity of nested submatrices, after Barnett; Sec. 5
// and Table 1: the "kernel degree estimation" stage).
//
// With the latent size unknown only d = H1 - H2 = k1 - k2 is known.  For a
// trial size k (k1' = k, k2' = k - d) and a unit-circle sample of either
// pass, the 1-D system A(k) = [C_{k-d}(e1) | -C_k(e2)] has a null vector
// exactly when k >= k1 (every solution of b1 u = b2 v is (k2 s, k1 s)), so
// its nullity is max(0, k - k1 + 1).  The test per trial size and sample is
//   s = lambda_min(G(k)) / lambda_max(G(k)),  G(k) = A(k)^H A(k),
// and G(k) is a principal submatrix of the Gram of the largest trial size:
// its entries are the same block-Toeplitz correlations (recover.hip), so one
// set of double-double correlations serves every candidate.
//
// k_size_probe: one wave per (candidate, pass, sample): G(k) from the
//   correlations (rounded to FP64), Householder tridiagonalisation, Sturm
//   multisection for the smallest and the largest eigenvalue.
// k_size_decide: one wave: per candidate the median over the 2S samples of
//   log10(max(s, 1e-13)); the estimate is the candidate with the largest
//   drop from the previous candidate's score (0 before the first); a largest
//   drop below 2 decades means no candidate made the systems singular.
#include "eigsmall.h"
#include "internal.h"

namespace cbp {

namespace {

constexpr double kSizeFloor = 1e-13;
constexpr double kSizeMinDrop = 2.0;

// Entry (r, c) of the Gram of trial sizes (n1 u taps, n2 v taps) from the
// correlations stored for the largest sizes (K2 u taps, K1 v taps):
// rho11[0..K2), rho22[0..K1), rho12[-(K1-1)..K2-1].
__device__ inline cdd trial_gram(const cdd* rho, int K1, int K2, int n1, int r, int c) {
  const bool ra = r < n1, ca = c < n1;
  const int pr = ra ? r : r - n1, pc = ca ? c : c - n1;   // index inside its block
  cdd v;
  if (ra == ca) {
    const int lag = pr - pc;
    v = rho[(ra ? 0 : K2) + (lag < 0 ? -lag : lag)];
    if (lag < 0) v.im = dd_neg(v.im);
  } else {
    // G12[p][q] = -rho12(p - q) (u index p, v index q); G21 = G12^H
    const int cross = K2 + K1 + (K1 - 1);
    v = ra ? rho[cross + pr - pc] : rho[cross + pc - pr];
    if (!ra) v.im = dd_neg(v.im);
    v = cdd_neg(v);
  }
  return v;
}

__global__ __launch_bounds__(SMALL_NT) void k_size_probe(batch_ref br, size_cands cands, double* ratios) {
  extern __shared__ __attribute__((aligned(16))) char sm_probe[];
  for_items<Q_SIZE_PROBE>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int S = d.S, K1 = d.k1, K2 = d.k2;
    const int NL = 2 * (K1 + K2) - 1;
    const int ci = item / (2 * S), rest = item - ci * 2 * S;
    const int pass = rest / S, j = rest - pass * S;
    const int k = cands.k1[ci];
    const int n2 = k, n1 = k - cands.d, n = n1 + n2;
    const int l = threadIdx.x;
    cdd* rho = (cdd*)sm_probe;
    small_ws w = small_probe_carve(sm_probe + (((size_t)NL * sizeof(cdd) + 15) & ~(size_t)15), n);
    for (int t = l; t < NL; t += SMALL_NT) rho[t] = d.corr[((size_t)pass * S + j) * NL + t];
    __syncthreads();
    for (int e = l; e < n * n; e += SMALL_NT) {
      const int r = e / n, c = e - r * n;
      const cdd g = trial_gram(rho, K1, K2, n1, r, c);
      w.A[e] = {g.re.hi, g.im.hi};
    }
    __syncthreads();
    const double r = small_extreme_ratio(w, n);
    if (l == 0) ratios[((size_t)ci * 2 + pass) * S + j] = r;
  });
}

// One wave: scores, drops and the decision.  ratios [ncand][2][S].
__global__ __launch_bounds__(SMALL_NT) void k_size_decide(size_cands cands, int S, const double* ratios,
                                                           cbp_size_result* out) {
  __shared__ double v[CBP_MAX_K][2 * CBP_MAX_S];
  __shared__ double score[CBP_MAX_K];
  const int l = threadIdx.x, nc = cands.n, m = 2 * S;
  if (l < nc) {
    // this lane's candidate: floored logs, insertion sort, median
    double* x = v[l];
    for (int t = 0; t < m; ++t) {
      const double r = ratios[(size_t)l * m + t];
      const double y = log10(fmax(r, kSizeFloor));
      int u = t;
      while (u > 0 && x[u - 1] > y) {
        x[u] = x[u - 1];
        --u;
      }
      x[u] = y;
    }
    score[l] = (m & 1) ? x[m / 2] : 0.5 * (x[m / 2 - 1] + x[m / 2]);
  }
  __syncthreads();
  if (l == 0) {
    int best = 0;
    double bestd = -1.0;
    for (int c = 0; c < nc; ++c) {
      const double dr = (c == 0 ? 0.0 : score[c - 1]) - score[c];
      out->score[c] = score[c];
      out->drop[c] = dr;
      out->cand[c] = cands.k1[c];
      if (dr > bestd) {
        bestd = dr;
        best = c;
      }
    }
    int flags = 0;
    if (!(bestd >= kSizeMinDrop)) {
      best = nc - 1;
      flags |= CBP_SIZE_NONE_SINGULAR;
    } else if (best == 0) {
      flags |= CBP_SIZE_FIRST_SINGULAR;
    }
    out->k1 = cands.k1[best];
    out->k2 = cands.k1[best] - cands.d;
    out->flags = flags;
    out->ncand = nc;
    out->samples = S;
  }
}

}  // namespace

size_t size_probe_lds_bytes(int nmax, int NLmax) {
  return (((size_t)NLmax * sizeof(cdd) + 15) & ~(size_t)15) + small_probe_lds_bytes(nmax);
}

void set_size_attrs() {
  hipFuncSetAttribute((const void*)k_size_probe, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)size_probe_lds_bytes(CBP_MAX_N, 2 * CBP_MAX_N - 1));
}

hipError_t launch_size_probe(const batch_ref& br, int grid, const size_cands& c, int nmax, int NLmax, double* ratios,
                             hipStream_t st) {
  const size_t lds = size_probe_lds_bytes(nmax, NLmax);
  hipLaunchKernelGGL(k_size_probe, dim3(grid), dim3(SMALL_NT), lds, st, br, c, ratios);
  return hipGetLastError();
}

hipError_t launch_size_decide(const size_cands& c, int S, const double* ratios, cbp_size_result* out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_size_decide, dim3(1), dim3(SMALL_NT), 0, st, c, S, ratios, out);
  return hipGetLastError();
}

}  // namespace cbp
