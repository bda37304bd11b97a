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
// accumulation.  Only the columns 0 and k2 of G are needed (every correlation
// is in them: rho11(l) = G[l][0], rho22(l) = G[k2+l][k2], rho12(l) = -G[l][k2]
// for l >= 0 and -conj(G[k2-l][0]) for l < 0), so only the four columns
// {0, k2, N, N + k2} of R = M^T M are formed: four 16 x 16 tiles (rows p of
// R in blocks of 16) whose first four columns are those (B's other columns
// are zero).  v_mfma_f64_16x16x4f64 takes A[i][k] from lane 16 k + i, B[k][j]
// from lane 16 k + j and leaves D[4 (lane / 16) + v][lane % 16] in
// accumulator v of each lane.
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GM64_RS = 5;      // row stride of the R column buffer (doubles)
constexpr int GM64_WAVES = 16;  // waves per workgroup: the rows of one item are split over them

__global__ __launch_bounds__(64 * GM64_WAVES) void k_gram_mfma64(batch_ref br) {
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
    double* Rc = (double*)sm_gm;                       // [64][GM64_RS]: R[p][{0, k2, N, N + k2}]
    double* sd = Rc + 64 * GM64_RS + 3;                // [4][P] staged re / im of e1 and -e2 (odd offset: 16-B aligned below)
    sd = (double*)(((size_t)sd + 15) & ~(size_t)15);
    // this lane's operands: A rows p = 16 pb + lane % 16 (four blocks pb),
    // B column jj = lane % 16 (columns 0..3 map to R's q in {0, k2, N, N + k2})
    const int i16 = lane & 15, kk = lane >> 4;
    mcol ca[4];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) ca[pb] = column_of(16 * pb + i16, k2, N);
    const int qs[4] = {0, k2, N, N + k2};
    const mcol cb = i16 < 4 ? column_of(qs[i16], k2, N) : mcol{-1, 0};
    v4d acc[4] = {};
    for (int ch = 0; ch < d.nch; ++ch) {
      const c64* e1 = base + ((size_t)(ch * 2 + 0) * S + j) * stride;
      const c64* e2 = base + ((size_t)(ch * 2 + 1) * S + j) * stride;
      for (int t = tid; t < P; t += 64 * GM64_WAVES) {
        const int i1 = t - GM_PAD_L;
        const c64 a = (i1 >= 0 && i1 < len1) ? e1[i1] : c64{0.0, 0.0};
        const c64 b = (i1 >= 0 && i1 < len2) ? e2[i1] : c64{0.0, 0.0};
        sd[0 * P + t] = a.re; sd[1 * P + t] = -b.re;
        sd[2 * P + t] = a.im; sd[3 * P + t] = -b.im;
      }
      __syncthreads();
      const double* pa[4];
#pragma unroll
      for (int pb = 0; pb < 4; ++pb) pa[pb] = ca[pb].arr >= 0 ? sd + ca[pb].arr * P + GM_PAD_L - ca[pb].shift : nullptr;
      const double* pbp = cb.arr >= 0 ? sd + cb.arr * P + GM_PAD_L - cb.shift : nullptr;
      // K = 4 rows per step: lane supplies row r0 + lane / 16; wave w takes
      // steps w, w + GM64_WAVES, ...
      for (int r0 = 4 * w; r0 < L; r0 += 4 * GM64_WAVES) {
        const int r = r0 + kk;
        const double bv = pbp ? pbp[r] : 0.0;
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) {
          const double av = pa[pb] ? pa[pb][r] : 0.0;
          acc[pb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[pb], 0, 0, 0);
        }
      }
      __syncthreads();  // staging buffers are rewritten for the next channel
    }
    // the waves' partial columns summed into Rc in wave order
    for (int ww = 0; ww < GM64_WAVES; ++ww) {
      if (w == ww && i16 < 4) {
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int p = 16 * pb + 4 * v + kk;   // D row 4 v + lane / 16, column lane % 16
            if (ww == 0) Rc[p * GM64_RS + i16] = acc[pb][v];
            else Rc[p * GM64_RS + i16] += acc[pb][v];
          }
      }
      __syncthreads();
    }
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
  });
}

}  // namespace

size_t gram_mfma_lds_bytes(int maxStride, int fmt) {
  const size_t P = (size_t)maxStride + GM_PAD;
  if (fmt == 2) return 64 * GM64_RS * sizeof(double) + 32 + 4 * P * sizeof(double);
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
