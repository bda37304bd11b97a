// Per-sample Gram matrices on the matrix cores (precision forms MFMA32,
// BF16 and MFMA64; the last at the end of this file).  G = A^H A for A = [C_k2(e1) | -C_k1(e2)] (the stacked convolution
// matrix of one sample) is a dense contraction over the L = len(e1) + k2 - 1
// rows of A.  In real form, with M = [Re A | Im A] (L x 2N, N = k1 + k2 <= 32,
// padded with zero columns to 64),
//   R = M^T M  (64 x 64),   Re G[p][q] = R[p][q] + R[N+p][N+q],
//                           Im G[p][q] = R[p][N+q] - R[N+p][q].
// R is accumulated in FP32 by v_mfma_f32_32x32x2_f32 (FP32 operands) or
// v_mfma_f32_32x32x16_bf16 (bfloat16 operands) over the three 32 x 32 tiles
// (0,0), (0,1), (1,1) of the symmetric R.  The operands are the FP64
// evaluations rounded to FP32 (nearest even), and for BF16 further to
// bfloat16 (nearest even on the 16 dropped bits).  Since A is block Toeplitz,
// G is determined by its first row and column in each block; those 2N - 1
// entries are written as the correlations the eigen-solver reads (low parts
// zero):  rho11(l) = G[l][0], rho22(l) = G[k2+l][k2], rho12(p - q) = -G[p][k2+q].
//
// One workgroup of four waves per (sample, pass); wave w takes the row steps
// w, w + 4, ...  The four partial tiles are added in LDS in wave order (a
// fixed order, so results do not depend on scheduling).
#include "internal.h"

#include <type_traits>

namespace cbp {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int GM_PAD_L = 32;   // zero entries before each staged vector (shifts up to 31)
constexpr int GM_PAD = 128;    // total zero padding per staged vector
constexpr int GM_RS = 65;      // row stride of the R tile buffer (floats)

// bfloat16 bits of a float, round to nearest even (finite inputs).
__device__ inline unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Column c of M for this lane: which staged array, which shift; -1 = zero column.
struct mcol {
  int arr;    // index of the staged array: part * 2 + frame
  int shift;  // row shift of the convolution column
};

__device__ inline mcol column_of(int c, int k2, int N) {
  if (c >= 2 * N) return {-1, 0};
  const int part = c >= N ? 1 : 0;
  const int cp = c - part * N;
  const int f = cp < k2 ? 0 : 1;
  return {part * 2 + f, f ? cp - k2 : cp};
}

// Items: (sample, pass).  FMT 0: FP32 operands; 1: bfloat16 operands.
template <int FMT>
__global__ __launch_bounds__(256) void k_gram_mfma(batch_ref br) {
  extern __shared__ __attribute__((aligned(16))) char sm_gm[];
  for_items<Q_GRAMM>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int S = d.S, k1 = d.k1, k2 = d.k2, N = k1 + k2, NL = 2 * N - 1;
    const int j = item % S, pass = item / S;
    const int len1 = pass ? d.H1 : d.W1, len2 = pass ? d.H2 : d.W2;
    const int L = len1 + k2 - 1;
    const int stride = pass ? d.Hmax : d.Wmax;
    const int P = stride + GM_PAD;
    const c64* base = pass ? d.ey : d.ex;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    float* Rl = (float*)sm_gm;                 // [64][GM_RS]
    char* stage = sm_gm + 64 * GM_RS * sizeof(float);
    float* sf = (float*)stage;                 // FMT 0: [4][P] floats
    unsigned short* sb = (unsigned short*)stage;  // FMT 1: [4][P] bfloat16 bits
    const mcol c0 = column_of(lane & 31, k2, N);
    const mcol c1 = column_of(32 + (lane & 31), k2, N);
    v16f acc00 = {}, acc01 = {}, acc11 = {};
    for (int ch = 0; ch < d.nch; ++ch) {
      const c64* e1 = base + ((size_t)(ch * 2 + 0) * S + j) * stride;
      const c64* e2 = base + ((size_t)(ch * 2 + 1) * S + j) * stride;
      // stage re / im of e1 and -e2, zero padded
      for (int t = tid; t < P; t += 256) {
        const int i1 = t - GM_PAD_L;
        const c64 a = (i1 >= 0 && i1 < len1) ? e1[i1] : c64{0.0, 0.0};
        const c64 b = (i1 >= 0 && i1 < len2) ? e2[i1] : c64{0.0, 0.0};
        const float ar = (float)a.re, ai = (float)a.im, br2 = -(float)b.re, bi = -(float)b.im;
        if (FMT == 0) {
          sf[0 * P + t] = ar; sf[1 * P + t] = br2;
          sf[2 * P + t] = ai; sf[3 * P + t] = bi;
        } else {
          sb[0 * P + t] = bf16_bits(ar); sb[1 * P + t] = bf16_bits(br2);
          sb[2 * P + t] = bf16_bits(ai); sb[3 * P + t] = bf16_bits(bi);
        }
      }
      __syncthreads();
      if (FMT == 0) {
        // K = 2 rows per step; lane supplies M[r0 + lane/32][column]
        const float* p0 = c0.arr >= 0 ? sf + c0.arr * P + GM_PAD_L - c0.shift : nullptr;
        const float* p1 = c1.arr >= 0 ? sf + c1.arr * P + GM_PAD_L - c1.shift : nullptr;
        for (int r0 = 2 * w; r0 < L; r0 += 8) {
          const int r = r0 + (lane >> 5);
          const float a0 = p0 ? p0[r] : 0.0f;
          const float a1 = p1 ? p1[r] : 0.0f;
          acc00 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, a0, acc00, 0, 0, 0);
          acc01 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, a1, acc01, 0, 0, 0);
          acc11 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, a1, acc11, 0, 0, 0);
        }
      } else {
        // K = 16 rows per step; lane supplies rows r0 + 8 (lane/32) + 0..7
        const unsigned short* p0 = c0.arr >= 0 ? sb + c0.arr * P + GM_PAD_L - c0.shift : nullptr;
        const unsigned short* p1 = c1.arr >= 0 ? sb + c1.arr * P + GM_PAD_L - c1.shift : nullptr;
        for (int r0 = 16 * w; r0 < L; r0 += 64) {
          const int r = r0 + 8 * (lane >> 5);
          v4u u0 = {0u, 0u, 0u, 0u}, u1 = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (p0) u0[e] = (unsigned int)p0[r + 2 * e] | ((unsigned int)p0[r + 2 * e + 1] << 16);
            if (p1) u1[e] = (unsigned int)p1[r + 2 * e] | ((unsigned int)p1[r + 2 * e + 1] << 16);
          }
          const v8bf b0 = __builtin_bit_cast(v8bf, u0);
          const v8bf b1 = __builtin_bit_cast(v8bf, u1);
          acc00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b0, b0, acc00, 0, 0, 0);
          acc01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b0, b1, acc01, 0, 0, 0);
          acc11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b1, b1, acc11, 0, 0, 0);
        }
      }
      __syncthreads();  // staging buffers are rewritten for the next channel
    }
    // sum the four waves' tiles into R, in wave order.  Accumulator v of lane
    // holds D[i][jj], jj = lane % 32, i = 8 (v / 4) + 4 (lane / 32) + v % 4.
    for (int ww = 0; ww < 4; ++ww) {
      if (w == ww) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), jj = lane & 31;
          if (ww == 0) {
            Rl[i * GM_RS + jj] = acc00[v];
            Rl[i * GM_RS + 32 + jj] = acc01[v];
            Rl[(32 + i) * GM_RS + 32 + jj] = acc11[v];
          } else {
            Rl[i * GM_RS + jj] += acc00[v];
            Rl[i * GM_RS + 32 + jj] += acc01[v];
            Rl[(32 + i) * GM_RS + 32 + jj] += acc11[v];
          }
        }
      }
      __syncthreads();
    }
    // correlations from the first row / column of each block of G
    auto R = [&](int a, int b) -> double {  // R is symmetric; the lower-left tile is not stored
      return a >= 32 && b < 32 ? (double)Rl[b * GM_RS + a] : (double)Rl[a * GM_RS + b];
    };
    for (int li = tid; li < NL; li += 256) {
      int p, q;
      double sg = 1.0;
      if (li < k2) { p = li; q = 0; }                               // rho11(l) = G[l][0]
      else if (li < k2 + k1) { p = k2 + (li - k2); q = k2; }        // rho22(l) = G[k2+l][k2]
      else {
        const int l = li - (k1 + k2) - (k1 - 1);                    // rho12(l) = -G[p][k2+q], p - q = l
        if (l >= 0) { p = l; q = k2; } else { p = 0; q = k2 - l; }
        sg = -1.0;
      }
      const double gre = R(p, q) + R(N + p, N + q);
      const double gim = R(p, N + q) - R(N + p, q);
      d.corr[((size_t)pass * S + j) * NL + li] = cdd{{sg * gre, 0.0}, {sg * gim, 0.0}};
    }
  });
}

// ---------------------------------------------------------------- FP64 matrix cores
// Precision form MFMA64: the Gram's correlations on v_mfma_f64_16x16x4f64
// from the FP64 evaluations themselves (no operand rounding), FP64
// accumulation.  Every correlation is in the columns 0 and k2 of G, so only
// the four columns {0, k2, N, N + k2} of R = M^T M are needed, and each of
// those columns has shift 0: with the staged arrays x_0 = Re e1, x_1 =
// -Re e2, x_2 = Im e1, x_3 = -Im e2 (x_a has k_a shifts: k2 for e1, k1 for
// e2),
//   R[(a, s)][(b, 0)] = c_ab(s) = sum_r x_a[r] x_b[r + s],  0 <= s < k_a,
// a lag correlation of two staged arrays.  With the rows split into blocks
// of 16, D_ab[i][j] = sum_m x_a[16 m + i] x_b[16 m + j] gives every lag at
// once: c_ab(l) = sum_{i<16} D_ab[i][i + l].  D_ab is formed in 16 x 16 tiles
// (columns j in [16 t, 16 t + 16)) by the matrix cores, K = 4 blocks (64
// rows) per instruction: A[i][k] = x_a[16 (m0 + k) + i] and B[k][jj] =
// x_b[16 (m0 + k) + 16 t + jj] are both the contiguous run x[64 step + lane]
// (shifted by 16 t for B).  For a < b one tile range serves c_ab and c_ba
// (c_ba(s) = c_ab(-s)); lags l in [-(k_b - 1), k_a - 1] need t from
// -ceil((k_b - 1) / 16) to floor((k_a + 14) / 16), for a = b t from 0.  That
// is 26 tiles for 2 <= k1, k2 <= 17 and at most 34 for k1 + k2 <= 32; each
// tile belongs to one wave for all rows, so no partial sums are combined and
// the result does not depend on scheduling.
// v_mfma_f64_16x16x4f64 takes A[i][k] from lane 16 k + i, B[k][j] from lane
// 16 k + j and leaves D[4 v + lane / 16][lane % 16] in accumulator v.
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GM64_RS = 5;      // row stride of the R column buffer (doubles)
constexpr int GM64_WAVES = 16;  // waves per workgroup; tile u of wave w is w + 16 u
constexpr int GM64_TPW = 3;     // tiles per wave at most

// Shifts of staged array a (e1 arrays: k2, e2 arrays: k1).
__host__ __device__ constexpr int gm64_k(int a, int k1, int k2) { return (a & 1) ? k1 : k2; }
__host__ __device__ constexpr int gm64_tlo(int a, int b, int k1, int k2) {
  return a == b ? 0 : -((gm64_k(b, k1, k2) + 14) >> 4);
}
__host__ __device__ constexpr int gm64_thi(int a, int k1, int k2) { return (gm64_k(a, k1, k2) + 14) >> 4; }
// Tiles of the (k1, k2) item: pairs a <= b in order (0,0), (0,1), .. (3,3).
__host__ __device__ constexpr int gm64_tiles(int k1, int k2) {
  int n = 0;
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b) n += gm64_thi(a, k1, k2) - gm64_tlo(a, b, k1, k2) + 1;
  return n;
}
constexpr int gm64_max_tiles() {
  int m = 0;
  for (int k1 = 1; k1 < 32; ++k1)
    for (int k2 = 1; k1 + k2 <= 32; ++k2) m = gm64_tiles(k1, k2) > m ? gm64_tiles(k1, k2) : m;
  return m;
}
constexpr int GM64_MAX_TILES = gm64_max_tiles();
static_assert(GM64_MAX_TILES <= GM64_WAVES * GM64_TPW, "tiles per wave");

// Tile index of (pair (a, b), a <= b, column block t) and its decode.
__device__ inline int gm64_tile_of(int a, int b, int t, int k1, int k2) {
  int n = 0;
  for (int aa = 0; aa < 4; ++aa)
    for (int bb = aa; bb < 4; ++bb) {
      const int lo = gm64_tlo(aa, bb, k1, k2);
      if (aa == a && bb == b) return n + t - lo;
      n += gm64_thi(aa, k1, k2) - lo + 1;
    }
  return -1;
}
struct gm64_tile { int a, b, t; };
__device__ inline gm64_tile gm64_decode(int tile, int k1, int k2) {
  int n = 0;
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b) {
      const int lo = gm64_tlo(a, b, k1, k2), cnt = gm64_thi(a, k1, k2) - lo + 1;
      if (tile < n + cnt) return {a, b, lo + tile - n};
      n += cnt;
    }
  return {0, 0, 0};
}

__global__ __launch_bounds__(64 * GM64_WAVES) void k_gram_mfma64(batch_ref br) {
  extern __shared__ __attribute__((aligned(16))) char sm_gm[];
  for_items<Q_GRAMM>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int S = d.S, k1 = d.k1, k2 = d.k2, N = k1 + k2, NL = 2 * N - 1;
    const int j = item % S, pass = item / S;
    const int len1 = pass ? d.H1 : d.W1, len2 = pass ? d.H2 : d.W2;
    const int stride = pass ? d.Hmax : d.Wmax;
    const int P = stride + GM_PAD;
    const c64* base = pass ? d.ey : d.ex;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double* Rc = (double*)sm_gm;                       // [64][GM64_RS]: R[p][{0, k2, N, N + k2}]
    double* sd = Rc + 64 * GM64_RS + 4;                // [4][P] staged x_0..x_3 (2592 B in: 16-B aligned)
    double* Dt = sd;                                   // [tiles][16][16], over the staging area once it is free
    // x_a is nonzero on [0, len_a): 16-row blocks up to the longer one, in steps of four
    const int nsteps = (max(len1, len2) + 63) >> 6;
    const int ntile = gm64_tiles(k1, k2);
    int ta[GM64_TPW], tb[GM64_TPW];
#pragma unroll
    for (int u = 0; u < GM64_TPW; ++u) {
      const gm64_tile tl = gm64_decode(w + GM64_WAVES * u, k1, k2);
      ta[u] = tl.a * P + GM_PAD_L + lane;
      tb[u] = tl.b * P + GM_PAD_L + 16 * tl.t + lane;
    }
    const int nt = __builtin_amdgcn_readfirstlane(ntile > w ? (ntile - w + GM64_WAVES - 1) / GM64_WAVES : 0);
    v4d acc[GM64_TPW] = {};
    // channel ch's entries t = tid + 1024 q (q < GM64_PF) are loaded into
    // registers while the previous channel's steps run, and staged after them
    constexpr int GM64_PF = 3;
    c64 fa[GM64_PF], fb[GM64_PF];
    auto fetch = [&](int ch) __attribute__((always_inline)) {
      const c64* e1 = base + ((size_t)(ch * 2 + 0) * S + j) * stride;
      const c64* e2 = base + ((size_t)(ch * 2 + 1) * S + j) * stride;
#pragma unroll
      for (int q = 0; q < GM64_PF; ++q) {
        const int i1 = tid + 64 * GM64_WAVES * q - GM_PAD_L;
        fa[q] = (i1 >= 0 && i1 < len1) ? e1[i1] : c64{0.0, 0.0};
        fb[q] = (i1 >= 0 && i1 < len2) ? e2[i1] : c64{0.0, 0.0};
      }
    };
    auto put = [&](int ch) __attribute__((always_inline)) {
      auto st4 = [&](int t, c64 a, c64 b) __attribute__((always_inline)) {
        sd[0 * P + t] = a.re; sd[1 * P + t] = -b.re;
        sd[2 * P + t] = a.im; sd[3 * P + t] = -b.im;
      };
#pragma unroll
      for (int q = 0; q < GM64_PF; ++q) {
        const int t = tid + 64 * GM64_WAVES * q;
        if (t < P) st4(t, fa[q], fb[q]);
      }
      const c64* e1 = base + ((size_t)(ch * 2 + 0) * S + j) * stride;
      const c64* e2 = base + ((size_t)(ch * 2 + 1) * S + j) * stride;
      for (int t = tid + 64 * GM64_WAVES * GM64_PF; t < P; t += 64 * GM64_WAVES) {
        const int i1 = t - GM_PAD_L;   // >= 0 here
        st4(t, i1 < len1 ? e1[i1] : c64{0.0, 0.0}, i1 < len2 ? e2[i1] : c64{0.0, 0.0});
      }
    };
    fetch(0);
    put(0);
    __syncthreads();
    for (int ch = 0; ch < d.nch; ++ch) {
      if (ch + 1 < d.nch) fetch(ch + 1);
      // the wave's tile count is fixed per loop, so the steps carry no branch
      auto steps = [&](auto ntc) __attribute__((always_inline)) {
        constexpr int n = decltype(ntc)::value;
#pragma unroll 2
        for (int st = 0; st < nsteps; ++st)
#pragma unroll
          for (int u = 0; u < n; ++u) {
            const double av = sd[ta[u] + 64 * st], bv = sd[tb[u] + 64 * st];
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
          }
      };
      if (nt >= 3) steps(std::integral_constant<int, 3>{});
      else if (nt == 2) steps(std::integral_constant<int, 2>{});
      else if (nt == 1) steps(std::integral_constant<int, 1>{});
      __syncthreads();  // staging buffers are rewritten for the next channel (or by the tiles)
      if (ch + 1 < d.nch) {
        put(ch + 1);
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u < GM64_TPW; ++u)
      if (u < nt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          Dt[(w + GM64_WAVES * u) * 256 + (4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc[u][v];
    __syncthreads();
    // R[p][qi] = c_{a(p), qi}(s(p)): a diagonal of the pair's tiles, i ascending
    if (tid < 4 * 2 * N) {
      const int p = tid >> 2, qi = tid & 3;
      const int part = p >= N ? 1 : 0, cp = p - part * N, f = cp < k2 ? 0 : 1;
      const int a = part * 2 + f, s = f ? cp - k2 : cp;
      const int lo = min(a, qi), hi = max(a, qi), l = a <= qi ? s : -s;
      const int t0 = gm64_tlo(lo, hi, k1, k2);
      const double* D = Dt + (size_t)gm64_tile_of(lo, hi, t0, k1, k2) * 256;
      double sum = 0.0;
      for (int i = 0; i < 16; ++i) {
        const int jj = i + l, t = (jj >> 4) - t0;   // jj >> 4 = floor(jj / 16)
        sum += D[t * 256 + i * 16 + (jj & 15)];
      }
      Rc[p * GM64_RS + qi] = sum;
    }
    __syncthreads();
    // G[p][c] for c in {0 (column 0), 1 (column k2)}
    auto G = [&](int p, int c) -> c64 {
      return c64{Rc[p * GM64_RS + c] + Rc[(N + p) * GM64_RS + 2 + c], Rc[p * GM64_RS + 2 + c] - Rc[(N + p) * GM64_RS + c]};
    };
    for (int li = tid; li < NL; li += 64 * GM64_WAVES) {
      c64 g;
      if (li < k2) g = G(li, 0);                                     // rho11(l) = G[l][0]
      else if (li < k2 + k1) g = G(k2 + (li - k2), 1);              // rho22(l) = G[k2+l][k2]
      else {
        const int l = li - (k1 + k2) - (k1 - 1);
        g = l >= 0 ? G(l, 1) : conj(G(k2 - l, 0));                   // G[l][k2] or G[0][k2-l]
        g = c64{-g.re, -g.im};                                       // rho12 = -G12
      }
      d.corr[((size_t)pass * S + j) * NL + li] = cdd{{g.re, 0.0}, {g.im, 0.0}};
    }
    // the next item's staging rewrites only the tiles' area, whose reads
    // ended at the barrier above; Rc is rewritten after two more barriers
  });
}

}  // namespace

size_t gram_mfma_lds_bytes(int maxStride, int fmt) {
  const size_t P = (size_t)maxStride + GM_PAD;
  if (fmt == 2)
    return 64 * GM64_RS * sizeof(double) + 32 + std::max<size_t>(4 * P, GM64_MAX_TILES * 256) * sizeof(double);
  return 64 * GM_RS * sizeof(float) + 4 * P * (fmt == 0 ? sizeof(float) : sizeof(unsigned short));
}

void set_gram_mfma_attrs() {
  hipFuncSetAttribute((const void*)k_gram_mfma<0>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  hipFuncSetAttribute((const void*)k_gram_mfma<1>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  hipFuncSetAttribute((const void*)k_gram_mfma64, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t launch_gram_mfma(const batch_ref& br, int grid, int fmt, int maxStride,
                            hipStream_t st) {
  prof_begin(PH_GRAM, st);
  if (fmt == 0)
    hipLaunchKernelGGL(k_gram_mfma<0>, dim3(grid), dim3(256), gram_mfma_lds_bytes(maxStride, 0), st, br);
  else if (fmt == 1)
    hipLaunchKernelGGL(k_gram_mfma<1>, dim3(grid), dim3(256), gram_mfma_lds_bytes(maxStride, 1), st, br);
  else
    hipLaunchKernelGGL(k_gram_mfma64, dim3(grid), dim3(64 * GM64_WAVES), gram_mfma_lds_bytes(maxStride, 2), st, br);
  prof_end(PH_GRAM, st);
  return hipGetLastError();
}

}  // namespace cbp
