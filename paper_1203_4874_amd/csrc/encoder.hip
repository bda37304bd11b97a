// The CBP encoder (Sec. 3, blur kernel selection; Sec. 4 eq. 1 without the
// sensor noise) and the multi-level 8-bit streams (Sec. 3, multi-level
// security).
//
// k_draw_pairs: one wave per frame draws the frame's kernel pair from the
//   counter-based generator Philox4x64-10 (Salmon, Moraes, Dror and Shaw,
//   SC 2011) -- entry e of kernel s, attempt a, is word e mod 4 of
//   Philox(counter (e / 4, s, a, 0), key (seed, frame)), u = ((w >> 11) + 1/2)
//   2^-53, normalised to sum 1 in entry order -- and redraws (a + 1) while at
//   some sample w_j of either evaluation order the Sylvester system of the two
//   kernel slices, [C_{k2-1}(p) | -C_{k1-1}(q)], has lambda_min / lambda_max
//   of its Gram below 1e-12 (the slices nearly share a root, so the pair is
//   not safely coprime).
// k_blur: B_s = L (x) K_s, full linear convolution of every channel with
//   both kernels, from LDS tiles of the latent (16 x 64 outputs per
//   workgroup, four rows per thread; each input column of the tile read once
//   per kernel column).
// k_quantize / k_dequantize: the 8-bit stream of a level without the b
//   least significant bits, q = clamp(rint(255 B), 0, 255) & (255 << b), and
//   the receiver's q / 255.
#include "eigsmall.h"
#include "internal.h"

namespace cbp {

namespace {

constexpr double kSylvMin = 1e-12;
constexpr int kMaxAttempts = 64;

// ---------------------------------------------------------------- Philox4x64-10
struct u64x4 {
  unsigned long long v[4];
};

__device__ inline u64x4 philox4x64(u64x4 c, unsigned long long k0, unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const unsigned long long hi0 = __umul64hi(M0, c.v[0]), lo0 = M0 * c.v[0];
    const unsigned long long hi1 = __umul64hi(M1, c.v[2]), lo1 = M1 * c.v[2];
    u64x4 o;
    o.v[0] = hi1 ^ c.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ c.v[3] ^ k1;
    o.v[3] = lo0;
    c = o;
  }
  return c;
}

// u_e of entry e of kernel `stream` (unnormalised, in (0, 1)).
__device__ inline double draw_entry(unsigned long long seed, unsigned long long frame, int stream, int attempt,
                                    int e) {
  u64x4 c;
  c.v[0] = (unsigned long long)(e >> 2);
  c.v[1] = (unsigned long long)stream;
  c.v[2] = (unsigned long long)attempt;
  c.v[3] = 0ull;
  const u64x4 w = philox4x64(c, seed, frame);
  const unsigned long long x = w.v[e & 3];
  return ((double)(x >> 11) + 0.5) * 0x1p-53;
}

// One kernel into K (LDS, k x k): entries in parallel, the sum in entry order
// on lane 0, then the division.
__device__ inline void draw_kernel(double* K, int k, unsigned long long seed, unsigned long long frame, int stream,
                                   int attempt, double* sum_slot) {
  for (int e = threadIdx.x; e < k * k; e += SMALL_NT) K[e] = draw_entry(seed, frame, stream, attempt, e);
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int e = 0; e < k * k; ++e) s += K[e];
    *sum_slot = s;
  }
  __syncthreads();
  const double s = *sum_slot;
  for (int e = threadIdx.x; e < k * k; e += SMALL_NT) K[e] = K[e] / s;
  __syncthreads();
}

// LDS of k_draw_pairs: two kernels, two slices, the correlations, a sum slot
// and the reduction workspace of order k1 + k2 - 2.
__host__ __device__ inline size_t draw_lds_bytes(int k1, int k2) {
  const int n = k1 + k2 - 2 > 1 ? k1 + k2 - 2 : 1;
  return (size_t)(k1 * k1 + k2 * k2 + 2) * sizeof(double) + 2 * (size_t)CBP_MAX_K * sizeof(c64) +
         (size_t)(2 * CBP_MAX_N) * sizeof(c64) + small_probe_lds_bytes(n) + 16;
}

__global__ __launch_bounds__(SMALL_NT) void k_draw_pairs(unsigned long long seed, long long frame0, int k1, int k2,
                                                          int S, double* K1s, double* K2s, int* attempts,
                                                          double* min_ratio) {
  extern __shared__ __attribute__((aligned(16))) char sm_draw[];
  const int f = blockIdx.x, l = threadIdx.x;
  const unsigned long long frame = (unsigned long long)(frame0 + f);
  double* K1 = (double*)sm_draw;
  double* K2 = K1 + k1 * k1;
  double* sum_slot = K2 + k2 * k2;
  c64* p = (c64*)(((size_t)(sum_slot + 2) + 15) & ~(size_t)15);
  c64* q = p + CBP_MAX_K;
  c64* rho = q + CBP_MAX_K;                     // [rho_pp (k1), rho_qq (k2), rho_pq (k1 + k2 - 1)]
  const int n1 = k2 - 1, n2 = k1 - 1, n = n1 + n2;
  small_ws w = small_probe_carve((char*)(rho + 2 * CBP_MAX_N), n > 1 ? n : 1);
  int found = -1;
  double worst = 1.0;
  for (int a = 0; a < kMaxAttempts && found < 0; ++a) {
    draw_kernel(K1, k1, seed, frame, 1, a, sum_slot);
    draw_kernel(K2, k2, seed, frame, 2, a, sum_slot);
    worst = 1.0;
    for (int pass = 0; pass < 2 && n > 0; ++pass)
      for (int j = 0; j < S; ++j) {
        // slices: pass 0 evaluates along y (a polynomial in x), pass 1 along x
        if (l < k1 + k2) {
          const bool first = l < k1;
          const int k = first ? k1 : k2, t = first ? l : l - k1;
          const double* K = first ? K1 : K2;
          c64 acc = {0.0, 0.0};
          for (int r = 0; r < k; ++r) {
            double sn, cs;
            sincospi(-2.0 * (double)((j * r) % S) / (double)S, &sn, &cs);
            const double kv = pass == 0 ? K[r * k + t] : K[t * k + r];
            acc = acc + c64{kv * cs, kv * sn};
          }
          (first ? p : q)[t] = acc;
        }
        __syncthreads();
        // correlations rho_pp(l) (l < k1), rho_qq(l) (l < k2), rho_pq(l), l in [-(n2 - 1), n1 - 1]
        for (int t = l; t < k1 + k2 + n - 1; t += SMALL_NT) {
          const c64* x;
          const c64* y;
          int lag, lx, ly;
          if (t < k1) { x = p; y = p; lag = t; lx = k1; ly = k1; }
          else if (t < k1 + k2) { x = q; y = q; lag = t - k1; lx = k2; ly = k2; }
          else { x = p; y = q; lag = t - (k1 + k2) - (n2 - 1); lx = k1; ly = k2; }
          c64 acc = {0.0, 0.0};
          for (int s0 = max(0, -lag); s0 < lx && s0 + lag < ly; ++s0) acc = acc + cmulc(x[s0], y[s0 + lag]);
          rho[t] = acc;
        }
        __syncthreads();
        for (int e = l; e < n * n; e += SMALL_NT) {
          const int r = e / n, c = e - r * n;
          const bool ra = r < n1, ca = c < n1;
          const int pr = ra ? r : r - n1, pc = ca ? c : c - n1;
          c64 v;
          if (ra == ca) {
            // rho_pp has k1 lags, rho_qq k2; longer lags are zero
            const int lag = pr - pc, al = lag < 0 ? -lag : lag;
            v = al < (ra ? k1 : k2) ? rho[(ra ? 0 : k1) + al] : c64{0.0, 0.0};
            if (lag < 0) v.im = -v.im;
          } else {
            const int cross = k1 + k2 + (n2 - 1);
            v = ra ? rho[cross + pr - pc] : conj(rho[cross + pc - pr]);
            v = c64{-v.re, -v.im};
          }
          w.A[e] = v;
        }
        __syncthreads();
        const double r = small_extreme_ratio(w, n);
        worst = fmin(worst, r);
        __syncthreads();
      }
    if (worst > kSylvMin) found = a;
  }
  for (int e = l; e < k1 * k1; e += SMALL_NT) K1s[(size_t)f * k1 * k1 + e] = K1[e];
  for (int e = l; e < k2 * k2; e += SMALL_NT) K2s[(size_t)f * k2 * k2 + e] = K2[e];
  if (l == 0) {
    attempts[f] = found;
    if (min_ratio) min_ratio[f] = worst;
  }
}

// ---------------------------------------------------------------- blur
constexpr int kTY = 16, kTX = 64;

// Items: (tile x, tile y, channel, stream).  B_s[y][x] = sum_{a,b} L[y-a][x-b] K_s[a][b].
template <typename T>
__global__ __launch_bounds__(256) void k_blur(const T* L, int64_t lp, int64_t lcs, int m, int n, int nch,
                                              const double* K1, int k1, const double* K2, int k2, T* B1,
                                              int64_t p1, int64_t cs1, T* B2, int64_t p2, int64_t cs2, int ntx,
                                              int nty1, int ntx1, int nty2, int ntx2) {
  __shared__ T Ks[CBP_MAX_K * CBP_MAX_K];
  __shared__ T tile[(kTY + CBP_MAX_K - 1) * (kTX + CBP_MAX_K - 1)];
  (void)ntx;
  const int per1 = nty1 * ntx1 * nch;
  int item = blockIdx.x;
  const int stream = item >= per1;
  if (stream) item -= per1;
  const int ntxs = stream ? ntx2 : ntx1, ntys = stream ? nty2 : nty1;
  const int tx0 = item % ntxs, rest = item / ntxs;
  const int ty0 = rest % ntys, ch = rest / ntys;
  const int k = stream ? k2 : k1;
  const double* K = stream ? K2 : K1;
  T* B = stream ? B2 : B1;
  const int64_t bp = stream ? p2 : p1, bcs = stream ? cs2 : cs1;
  const int H = m + k - 1, W = n + k - 1;
  const int y0 = ty0 * kTY, x0 = tx0 * kTX;
  const int tw = kTX + k - 1, th = kTY + k - 1;
  for (int e = threadIdx.x; e < k * k; e += 256) Ks[e] = (T)K[e];
  const T* Lc = L + (int64_t)ch * lcs;
  for (int e = threadIdx.x; e < th * tw; e += 256) {
    const int i = e / tw, jj = e - i * tw;
    const int y = y0 - (k - 1) + i, x = x0 - (k - 1) + jj;
    tile[e] = (y >= 0 && y < m && x >= 0 && x < n) ? Lc[(int64_t)y * lp + x] : T(0);
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, tyg = threadIdx.x >> 6;   // 64 columns x 4 row groups of 4 rows
  T acc[4] = {T(0), T(0), T(0), T(0)};
  for (int b = 0; b < k; ++b) {
    // the tile column this thread's outputs read for kernel column b: rows
    // 4 tyg + i, i < k + 3; output row r takes row i with kernel row
    // a = r + k - 1 - i (each tile value read once per kernel column)
    const T* col = tile + (4 * tyg) * tw + (tx - b + k - 1);
    for (int i = 0; i < k + 3; ++i) {
      const T v = col[i * tw];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = r + k - 1 - i;
        if (a >= 0 && a < k) acc[r] += v * Ks[a * k + b];
      }
    }
  }
  T* Bc = B + (int64_t)ch * bcs;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int y = y0 + 4 * tyg + r, x = x0 + tx;
    if (y < H && x < W) Bc[(int64_t)y * bp + x] = acc[r];
  }
}

// ---------------------------------------------------------------- 8-bit streams
template <typename T>
__global__ void k_quantize(const T* src, int64_t sp, int64_t scs, unsigned char* dst, int64_t dp, int64_t dcs,
                           int H, int W, int nch, int drop) {
  const int64_t total = (int64_t)H * W * nch;
  const unsigned int mask = (0xFFu << drop) & 0xFFu;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(e % W);
    const int64_t r = e / W;
    const int y = (int)(r % H), c = (int)(r / H);
    const T v = rint(src[(int64_t)c * scs + (int64_t)y * sp + x] * T(255));
    const T cl = v < T(0) ? T(0) : (v > T(255) ? T(255) : v);
    dst[(int64_t)c * dcs + (int64_t)y * dp + x] = (unsigned char)((unsigned int)cl & mask);
  }
}

template <typename T>
__global__ void k_dequantize(const unsigned char* src, int64_t sp, int64_t scs, T* dst, int64_t dp, int64_t dcs,
                             int H, int W, int nch) {
  const int64_t total = (int64_t)H * W * nch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(e % W);
    const int64_t r = e / W;
    const int y = (int)(r % H), c = (int)(r / H);
    dst[(int64_t)c * dcs + (int64_t)y * dp + x] = (T)src[(int64_t)c * scs + (int64_t)y * sp + x] / T(255);
  }
}

}  // namespace

hipError_t launch_draw_pairs(unsigned long long seed, long long frame0, int nframes, int k1, int k2, int S,
                             double* K1s, double* K2s, int* attempts, double* min_ratio, hipStream_t st) {
  const size_t lds = draw_lds_bytes(k1, k2);
  hipLaunchKernelGGL(k_draw_pairs, dim3(nframes), dim3(SMALL_NT), lds, st, seed, frame0, k1, k2, S, K1s, K2s,
                     attempts, min_ratio);
  return hipGetLastError();
}

size_t draw_pairs_lds_bytes(int k1, int k2) { return draw_lds_bytes(k1, k2); }

void set_encoder_attrs() {
  hipFuncSetAttribute((const void*)k_draw_pairs, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)draw_lds_bytes(CBP_MAX_K, CBP_MAX_K));
}

template <typename T>
hipError_t launch_blur(const T* L, int64_t lp, int64_t lcs, int m, int n, int nch, const double* K1, int k1,
                       const double* K2, int k2, T* B1, int64_t p1, int64_t cs1, T* B2, int64_t p2, int64_t cs2,
                       hipStream_t st) {
  const int nty1 = (m + k1 - 1 + kTY - 1) / kTY, ntx1 = (n + k1 - 1 + kTX - 1) / kTX;
  const int nty2 = (m + k2 - 1 + kTY - 1) / kTY, ntx2 = (n + k2 - 1 + kTX - 1) / kTX;
  const int grid = (nty1 * ntx1 + nty2 * ntx2) * nch;
  hipLaunchKernelGGL(k_blur<T>, dim3(grid), dim3(256), 0, st, L, lp, lcs, m, n, nch, K1, k1, K2, k2, B1, p1, cs1,
                     B2, p2, cs2, 0, nty1, ntx1, nty2, ntx2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_quantize(const T* src, int64_t sp, int64_t scs, unsigned char* dst, int64_t dp, int64_t dcs, int H,
                           int W, int nch, int drop, hipStream_t st) {
  const int64_t total = (int64_t)H * W * nch;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_quantize<T>, dim3(grid), dim3(256), 0, st, src, sp, scs, dst, dp, dcs, H, W, nch, drop);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dequantize(const unsigned char* src, int64_t sp, int64_t scs, T* dst, int64_t dp, int64_t dcs,
                             int H, int W, int nch, hipStream_t st) {
  const int64_t total = (int64_t)H * W * nch;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_dequantize<T>, dim3(grid), dim3(256), 0, st, src, sp, scs, dst, dp, dcs, H, W, nch);
  return hipGetLastError();
}

template hipError_t launch_blur<float>(const float*, int64_t, int64_t, int, int, int, const double*, int,
                                       const double*, int, float*, int64_t, int64_t, float*, int64_t, int64_t,
                                       hipStream_t);
template hipError_t launch_blur<double>(const double*, int64_t, int64_t, int, int, int, const double*, int,
                                        const double*, int, double*, int64_t, int64_t, double*, int64_t, int64_t,
                                        hipStream_t);
template hipError_t launch_quantize<float>(const float*, int64_t, int64_t, unsigned char*, int64_t, int64_t, int, int,
                                           int, int, hipStream_t);
template hipError_t launch_quantize<double>(const double*, int64_t, int64_t, unsigned char*, int64_t, int64_t, int,
                                            int, int, int, hipStream_t);
template hipError_t launch_dequantize<float>(const unsigned char*, int64_t, int64_t, float*, int64_t, int64_t, int,
                                             int, int, hipStream_t);
template hipError_t launch_dequantize<double>(const unsigned char*, int64_t, int64_t, double*, int64_t, int64_t, int,
                                              int, int, hipStream_t);

}  // namespace cbp
