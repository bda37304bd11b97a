// The learned form's network: a 32 -> 128 -> 128 -> 2 MLP with ReLU, BF16
// weights and activations on the matrix cores (v_mfma_f32_32x32x16_bf16) with
// FP32 accumulation, FP32 biases, FP32 master weights and Adam moments for
// training.  It reads each sample's Gram spectrum and predicts a confidence
// weight w = clip(softplus(o1), 1e-3, 1e3) and a Tikhonov strength
// tau = exp(clip(o2, -30, 5)); the paper has no counterpart of this form.
//
// Layouts (row-major; "bf16" = bfloat16 bits, round to nearest even):
//   parameters, FP32, packed: W1 [128][32], b1 [128], W2 [128][128], b2 [128],
//                             W3 [2][128], b3 [2]                 (MLP_NPARAM)
//   inference blob: header (4 x uint32: magic, version, 32, 128), then bf16
//                   W1, W2, W3 and FP32 b1, b2, b3                 (mlp_blob)
//   features X [n][32] FP32; outputs [n][2] FP32 (o1, o2).
//
// Matrix-core tiles: a 32 x 32 FP32 tile D = A B^T with A [32][K], B [32][K]
// (k contiguous in LDS).  Lane l supplies row l % 32 of A (and of B) at
// k = k0 + 8 (l / 32) .. + 7; accumulator v of lane l is
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
#include "mlp.h"

#include "internal.h"

namespace cbp {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ inline unsigned short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// D += A B^T over K (a multiple of 16) for one wave; A, B: 32 rows with row
// stride lda / ldb (elements), k contiguous, 16-byte aligned rows.
__device__ inline void tile_abt(const unsigned short* A, int lda, const unsigned short* B, int ldb, int K,
                                v16f& acc) {
  const int l = threadIdx.x & 63;
  const unsigned short* a = A + (size_t)(l & 31) * lda + 8 * (l >> 5);
  const unsigned short* b = B + (size_t)(l & 31) * ldb + 8 * (l >> 5);
  for (int k0 = 0; k0 < K; k0 += 16) {
    const v4u ua = *(const v4u*)(a + k0);
    const v4u ub = *(const v4u*)(b + k0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, ua), __builtin_bit_cast(v8bf, ub), acc,
                                                  0, 0, 0);
  }
}

__device__ inline int tile_row(int v) { return 8 * (v >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (v & 3); }
__device__ inline int tile_col() { return threadIdx.x & 31; }

constexpr int RB = 64;          // rows per workgroup in the row-blocked kernels
constexpr int LD1 = MLP_FEAT + 8;    // LDS row strides (bf16), padded against bank conflicts
constexpr int LDH = MLP_HIDDEN + 8;

// ------------------------------------------------------------------ forward
// One workgroup (4 waves) per block of 64 rows.  Layer 1 and 2 on the matrix
// cores; the 2-output head on the vector units in FP32.  With train != 0 the
// activations are kept for the backward pass: H1, H2 (bf16, [n][128]) and the
// pre-activation signs.
struct fwd_args {
  const float* X;
  int n;
  const unsigned short* W1;  // bf16 [128][32]
  const unsigned short* W2;  // bf16 [128][128]
  const float* W3;           // FP32 [2][128] (the head stays FP32)
  const float* b1;
  const float* b2;
  const float* b3;
  float* out;                // [n][2]
  unsigned short* H1;        // [n][128] (train)
  unsigned short* H2;        // [n][128] (train)
};

// LDS of one 64-row block.
struct fwd_lds {
  unsigned short xs[RB * LD1];
  unsigned short w1s[MLP_HIDDEN * LD1];
  unsigned short hs[RB * LDH];
  unsigned short w2s[MLP_HIDDEN * LDH];
  float h2f[RB][MLP_HIDDEN + 1];
  float out[RB][MLP_OUT];
};

// Forward of rows [0, nrows) of X (nrows <= 64) into L.out; with H1 / H2 not
// NULL the bf16 activations are stored there (row-major, 128 per row).
__device__ inline void mlp_block(fwd_lds& L, const float* X, int nrows, const unsigned short* W1,
                                 const unsigned short* W2, const float* W3, const float* b1, const float* b2,
                                 const float* b3, unsigned short* H1, unsigned short* H2) {
  const int tid = threadIdx.x, w = tid >> 6;
  for (int e = tid; e < RB * MLP_FEAT; e += 256) {
    const int r = e / MLP_FEAT, f = e % MLP_FEAT;
    L.xs[r * LD1 + f] = r < nrows ? to_bf16(X[(size_t)r * MLP_FEAT + f]) : (unsigned short)0;
  }
  for (int e = tid; e < MLP_HIDDEN * MLP_FEAT; e += 256) L.w1s[(e / MLP_FEAT) * LD1 + e % MLP_FEAT] = W1[e];
  for (int e = tid; e < MLP_HIDDEN * MLP_HIDDEN; e += 256) L.w2s[(e / MLP_HIDDEN) * LDH + e % MLP_HIDDEN] = W2[e];
  __syncthreads();
  // layer 1: 64 x 128 = 2 x 4 tiles of 32 x 32 over the 4 waves
  for (int t = w; t < 8; t += 4) {
    const int ti = t >> 2, tj = t & 3;
    v16f acc = {};
    tile_abt(L.xs + ti * 32 * LD1, LD1, L.w1s + tj * 32 * LD1, LD1, MLP_FEAT, acc);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = ti * 32 + tile_row(v), h = tj * 32 + tile_col();
      L.hs[r * LDH + h] = to_bf16(fmaxf(acc[v] + b1[h], 0.0f));
    }
  }
  __syncthreads();
  if (H1)
    for (int e = tid; e < RB * MLP_HIDDEN; e += 256) {
      const int r = e / MLP_HIDDEN, h = e % MLP_HIDDEN;
      if (r < nrows) H1[(size_t)r * MLP_HIDDEN + h] = L.hs[r * LDH + h];
    }
  // layer 2
  for (int t = w; t < 8; t += 4) {
    const int ti = t >> 2, tj = t & 3;
    v16f acc = {};
    tile_abt(L.hs + ti * 32 * LDH, LDH, L.w2s + tj * 32 * LDH, LDH, MLP_HIDDEN, acc);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = ti * 32 + tile_row(v), h = tj * 32 + tile_col();
      L.h2f[r][h] = from_bf16(to_bf16(fmaxf(acc[v] + b2[h], 0.0f)));
    }
  }
  __syncthreads();
  if (H2)
    for (int e = tid; e < RB * MLP_HIDDEN; e += 256) {
      const int r = e / MLP_HIDDEN, h = e % MLP_HIDDEN;
      if (r < nrows) H2[(size_t)r * MLP_HIDDEN + h] = to_bf16(L.h2f[r][h]);
    }
  // head: 2 outputs per row, 128-term FP32 dot products on the vector units
  if (tid < MLP_OUT * RB) {
    const int r = tid >> 1, o = tid & 1;
    float sacc = b3[o];
    for (int h = 0; h < MLP_HIDDEN; ++h) sacc = fmaf(L.h2f[r][h], W3[o * MLP_HIDDEN + h], sacc);
    L.out[r][o] = sacc;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_forward(fwd_args a) {
  __shared__ __attribute__((aligned(16))) fwd_lds L;
  const int r0 = blockIdx.x * RB;
  const int nrows = min(RB, a.n - r0);
  mlp_block(L, a.X + (size_t)r0 * MLP_FEAT, nrows, a.W1, a.W2, a.W3, a.b1, a.b2, a.b3,
            a.H1 ? a.H1 + (size_t)r0 * MLP_HIDDEN : nullptr, a.H2 ? a.H2 + (size_t)r0 * MLP_HIDDEN : nullptr);
  if (threadIdx.x < MLP_OUT * RB) {
    const int r = threadIdx.x >> 1, o = threadIdx.x & 1;
    if (r < nrows) a.out[(size_t)(r0 + r) * MLP_OUT + o] = L.out[r][o];
  }
}

// The learned form inside a deblurring call: per frame, the 2S samples'
// features (written by the eigen-solve kernel) through the network, then
//   wts[j] = w of pass-X sample j, wts[S + i] = w of pass-Y sample i,
//   wts[2S] = tau = median of the 2S values tau_j (mean of the middle two).
// Items: one per frame.
__global__ __launch_bounds__(256) void k_mlp_frames(batch_ref br, const mlp_blob* blob) {
  __shared__ __attribute__((aligned(16))) fwd_lds L;
  __shared__ double tj[64];
  __shared__ double mid[2];
  for_items<Q_FINALIZE>(br, [&](const frame_desc& d, int) __attribute__((always_inline)) {
    const int n = 2 * d.S;
    const int t = threadIdx.x;
    // a blob whose header is not this network's: unit weights and tau = 0
    // (the learned assembly then reduces to the plain one) and a flag
    if (blob->magic != MLP_MAGIC || blob->version != MLP_VERSION || blob->feat != MLP_FEAT ||
        blob->hidden != MLP_HIDDEN) {
      if (t < n) d.wts[t] = 1.0;
      if (t == 0) {
        d.wts[n] = 0.0;
        if (d.diag) atomicOr(&d.diag->flags, CBP_DIAG_BAD_NETWORK);
      }
      return;
    }
    mlp_block(L, d.feat, n, blob->W1, blob->W2, blob->W3, blob->b1, blob->b2, blob->b3, nullptr, nullptr);
    if (t < n) {
      const double o1 = L.out[t][0], o2 = L.out[t][1];
      const double sp = o1 > 30.0 ? o1 : log1p(exp(o1));
      d.wts[t] = fmin(fmax(sp, 1e-3), 1e3);
      tj[t] = exp(fmin(fmax(o2, -30.0), 5.0));
    }
    __syncthreads();
    if (t < n) {
      const double v = tj[t];
      int rank = 0;
      for (int u = 0; u < n; ++u) rank += (tj[u] < v) || (tj[u] == v && u < t);
      if (rank == n / 2 - 1) mid[0] = v;
      if (rank == n / 2) mid[1] = v;
    }
    __syncthreads();
    if (t == 0) d.wts[n] = 0.5 * (mid[0] + mid[1]);
  });
}

// ------------------------------------------------------------------ loss and head backward
// Per row: o = (o1, o2), loss_r = (log softplus(o1) - t1)^2 + (o2 - t2)^2,
// dO = d(mean loss)/dO; dH2 = dO W3, dZ2 = dH2 * [H2 > 0] (bf16, [n][128]).
// Per-block partial sums of the loss, dW3 and db3 (fixed order).
__global__ __launch_bounds__(256) void k_mlp_loss(const float* out, const float* T, int n, const float* W3,
                                                  const unsigned short* H2, unsigned short* dZ2, float* part) {
  __shared__ float dos[RB][2];
  __shared__ float red[256];
  const int tid = threadIdx.x, r0 = blockIdx.x * RB;
  float lsum = 0.0f;
  if (tid < RB) {
    const int r = r0 + tid;
    float d1 = 0.0f, d2 = 0.0f;
    if (r < n) {
      const float o1 = out[(size_t)r * 2], o2 = out[(size_t)r * 2 + 1];
      const float sp = o1 > 20.0f ? o1 : log1pf(expf(o1));
      const float sg = 1.0f / (1.0f + expf(-o1));
      const float r1 = logf(sp) - T[(size_t)r * 2], r2 = o2 - T[(size_t)r * 2 + 1];
      lsum = r1 * r1 + r2 * r2;
      d1 = 2.0f * r1 / (float)n * sg / sp;
      d2 = 2.0f * r2 / (float)n;
    }
    dos[tid][0] = d1;
    dos[tid][1] = d2;
  }
  __syncthreads();
  for (int e = tid; e < RB * MLP_HIDDEN; e += 256) {
    const int rr = e / MLP_HIDDEN, h = e % MLP_HIDDEN, r = r0 + rr;
    if (r < n) {
      const unsigned short hb = H2[(size_t)r * MLP_HIDDEN + h];
      const float g = dos[rr][0] * W3[h] + dos[rr][1] * W3[MLP_HIDDEN + h];
      dZ2[(size_t)r * MLP_HIDDEN + h] = from_bf16(hb) > 0.0f ? to_bf16(g) : (unsigned short)0;
    }
  }
  // partials: [0] loss, [1 .. 256] dW3, [257, 258] db3
  float* p = part + (size_t)blockIdx.x * (2 + 2 * MLP_HIDDEN + 1);
  red[tid] = tid < RB ? lsum : 0.0f;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) p[0] = red[0];
  // dW3[o][h] = sum_r dO[r][o] H2[r][h]
  {
    const int o = tid >> 7, h = tid & 127;
    float s = 0.0f;
    for (int rr = 0; rr < RB; ++rr)
      if (r0 + rr < n) s = fmaf(dos[rr][o], from_bf16(H2[(size_t)(r0 + rr) * MLP_HIDDEN + h]), s);
    p[1 + o * MLP_HIDDEN + h] = s;
  }
  if (tid < 2) {
    float s = 0.0f;
    for (int rr = 0; rr < RB; ++rr) s += dos[rr][tid];
    p[1 + 2 * MLP_HIDDEN + tid] = s;
  }
}

// ------------------------------------------------------------------ row-blocked backward
// dZ1 = (dZ2 W2) * [H1 > 0] for a block of 64 rows (bf16), using W2^T.
__global__ __launch_bounds__(256) void k_mlp_back_h1(const unsigned short* dZ2, const unsigned short* W2t,
                                                     const unsigned short* H1, int n, unsigned short* dZ1) {
  __shared__ __attribute__((aligned(16))) unsigned short ds_[RB * LDH];
  __shared__ __attribute__((aligned(16))) unsigned short wt[MLP_HIDDEN * LDH];
  const int tid = threadIdx.x, w = tid >> 6, r0 = blockIdx.x * RB;
  for (int e = tid; e < RB * MLP_HIDDEN; e += 256) {
    const int r = e / MLP_HIDDEN, h = e % MLP_HIDDEN;
    ds_[r * LDH + h] = r0 + r < n ? dZ2[(size_t)(r0 + r) * MLP_HIDDEN + h] : (unsigned short)0;
  }
  for (int e = tid; e < MLP_HIDDEN * MLP_HIDDEN; e += 256) wt[(e / MLP_HIDDEN) * LDH + e % MLP_HIDDEN] = W2t[e];
  __syncthreads();
  for (int t = w; t < 8; t += 4) {
    const int ti = t >> 2, tj = t & 3;
    v16f acc = {};
    tile_abt(ds_ + ti * 32 * LDH, LDH, wt + tj * 32 * LDH, LDH, MLP_HIDDEN, acc);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = r0 + ti * 32 + tile_row(v), h = tj * 32 + tile_col();
      if (r < n) {
        const bool on = from_bf16(H1[(size_t)r * MLP_HIDDEN + h]) > 0.0f;
        dZ1[(size_t)r * MLP_HIDDEN + h] = on ? to_bf16(acc[v]) : (unsigned short)0;
      }
    }
  }
}

// ------------------------------------------------------------------ weight gradients
// G[M][N] partial over a chunk of rows: G[i][j] = sum_r A[r][i] B[r][j], with
// A [n][M] and B [n][N] row-major over r, each either bf16 (Ab / Bb) or FP32
// rounded to bf16 on load (Af / Bf).  One wave per (32 x 32 tile of G, chunk
// of 256 rows); the chunk is transposed into LDS so the matrix-core operands
// have r contiguous.  Partials [chunk][M][N] FP32.
struct wgrad_args {
  const unsigned short* Ab;
  const float* Af;
  int M;
  const unsigned short* Bb;
  const float* Bf;
  int N;
  int n;
  float* part;
};

__global__ __launch_bounds__(64) void k_mlp_wgrad(wgrad_args g) {
  constexpr int CH = 256;
  __shared__ __attribute__((aligned(16))) unsigned short at[32 * (CH + 8)];
  __shared__ __attribute__((aligned(16))) unsigned short bt[32 * (CH + 8)];
  const int tilesN = g.N / 32;
  const int ti = blockIdx.x / tilesN, tj = blockIdx.x % tilesN;
  const int c = blockIdx.y, rbase = c * CH;
  const int l = threadIdx.x;
  for (int e = l; e < 32 * CH; e += 64) {
    const int rr = e / 32, i = e % 32, r = rbase + rr;
    unsigned short va = 0, vb = 0;
    if (r < g.n) {
      const size_t ia = (size_t)r * g.M + ti * 32 + i, ib = (size_t)r * g.N + tj * 32 + i;
      va = g.Ab ? g.Ab[ia] : to_bf16(g.Af[ia]);
      vb = g.Bb ? g.Bb[ib] : to_bf16(g.Bf[ib]);
    }
    at[i * (CH + 8) + rr] = va;
    bt[i * (CH + 8) + rr] = vb;
  }
  __syncthreads();
  v16f acc = {};
  tile_abt(at, CH + 8, bt, CH + 8, CH, acc);
  float* p = g.part + (size_t)c * g.M * g.N;
#pragma unroll
  for (int v = 0; v < 16; ++v) p[(size_t)(ti * 32 + tile_row(v)) * g.N + tj * 32 + tile_col()] = acc[v];
}

// Bias gradient partials: db[j] over a chunk of 256 rows of D [n][N] (bf16).
__global__ __launch_bounds__(128) void k_mlp_bgrad(const unsigned short* D, int N, int n, float* part) {
  const int j = threadIdx.x, c = blockIdx.x;
  float s = 0.0f;
  for (int r = c * 256; r < min(n, (c + 1) * 256); ++r) s += from_bf16(D[(size_t)r * N + j]);
  part[(size_t)c * N + j] = s;
}

// Sum partials over chunks in chunk order into g (FP32).
__global__ void k_mlp_reduce(const float* part, int nchunk, int len, int stride, float* g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.0f;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * stride + i];
  g[i] = s;
}

// Adam on the FP32 master weights, then the bf16 copies (W1, W2, W2^T) and
// the FP32 head.
__global__ void k_mlp_adam(float* p, float* m, float* v, const float* g, int np, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_mlp_quantise(const float* p, unsigned short* W1, unsigned short* W2, unsigned short* W2t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < MLP_HIDDEN * MLP_FEAT) W1[i] = to_bf16(p[MLP_OFF_W1 + i]);
  if (i < MLP_HIDDEN * MLP_HIDDEN) {
    const unsigned short q = to_bf16(p[MLP_OFF_W2 + i]);
    W2[i] = q;
    W2t[(i % MLP_HIDDEN) * MLP_HIDDEN + i / MLP_HIDDEN] = q;
  }
}

__global__ void k_mlp_scale(float* x, float f) { x[0] *= f; }

__global__ void k_mlp_zero2(float* a, float* b, int np) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) { a[i] = 0.0f; b[i] = 0.0f; }
}

// The inference blob from the FP32 master weights.
__global__ void k_mlp_export(const float* p, mlp_blob* b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) { b->magic = MLP_MAGIC; b->version = MLP_VERSION; b->feat = MLP_FEAT; b->hidden = MLP_HIDDEN; }
  if (i < MLP_HIDDEN * MLP_FEAT) b->W1[i] = to_bf16(p[MLP_OFF_W1 + i]);
  if (i < MLP_HIDDEN * MLP_HIDDEN) b->W2[i] = to_bf16(p[MLP_OFF_W2 + i]);
  if (i < MLP_OUT * MLP_HIDDEN) b->W3[i] = p[MLP_OFF_W3 + i];
  if (i < MLP_HIDDEN) { b->b1[i] = p[MLP_OFF_B1 + i]; b->b2[i] = p[MLP_OFF_B2 + i]; }
  if (i < MLP_OUT) b->b3[i] = p[MLP_OFF_B3 + i];
}

}  // namespace

// ------------------------------------------------------------------ host side
namespace {

struct state_view {
  float *p, *m, *v, *g;                 // MLP_NPARAM each
  unsigned short *W1, *W2, *W2t;        // bf16 copies
  unsigned short *H1, *H2, *dZ2, *dZ1;  // [rows][128]
  float* out;                           // [rows][2]
  float* part;                          // partial sums
};

size_t part_floats(int rows) {
  const size_t nb = (rows + RB - 1) / RB, nc = (rows + 255) / 256;
  const size_t a = nb * (2 + 2 * MLP_HIDDEN + 1);
  const size_t b = nc * MLP_HIDDEN * MLP_HIDDEN;
  return a > b ? a : b;
}

state_view carve(void* base, int rows) {
  char* c = (char*)base;
  auto take = [&](size_t bytes) { char* at = c; c += (bytes + 255) & ~(size_t)255; return at; };
  state_view s;
  s.p = (float*)take(MLP_NPARAM * 4);
  s.m = (float*)take(MLP_NPARAM * 4);
  s.v = (float*)take(MLP_NPARAM * 4);
  s.g = (float*)take(MLP_NPARAM * 4);
  s.W1 = (unsigned short*)take(MLP_HIDDEN * MLP_FEAT * 2);
  s.W2 = (unsigned short*)take(MLP_HIDDEN * MLP_HIDDEN * 2);
  s.W2t = (unsigned short*)take(MLP_HIDDEN * MLP_HIDDEN * 2);
  s.H1 = (unsigned short*)take((size_t)rows * MLP_HIDDEN * 2);
  s.H2 = (unsigned short*)take((size_t)rows * MLP_HIDDEN * 2);
  s.dZ2 = (unsigned short*)take((size_t)rows * MLP_HIDDEN * 2);
  s.dZ1 = (unsigned short*)take((size_t)rows * MLP_HIDDEN * 2);
  s.out = (float*)take((size_t)rows * 2 * 4);
  s.part = (float*)take(part_floats(rows) * 4);
  return s;
}

size_t carve_bytes(int rows) {
  state_view s = carve(nullptr, rows);
  return (size_t)((char*)s.part - (char*)nullptr) + ((part_floats(rows) * 4 + 255) & ~(size_t)255);
}

}  // namespace

size_t mlp_state_bytes(int rows) { return carve_bytes(rows); }

hipError_t launch_mlp_frames(const batch_ref& br, int grid, const void* blob,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_frames, dim3(grid), dim3(256), 0, st, br, (const mlp_blob*)blob);
  return hipGetLastError();
}

hipError_t mlp_forward_blob(const void* blob, const float* X, int n, float* out, hipStream_t st) {
  const mlp_blob* b = (const mlp_blob*)blob;
  fwd_args a = {X, n, b->W1, b->W2, b->W3, b->b1, b->b2, b->b3, out, nullptr, nullptr};
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + RB - 1) / RB), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t mlp_set_params(void* state, int rows, const float* params, hipStream_t st) {
  const state_view s = carve(state, rows);
  const hipError_t e = hipMemcpyAsync(s.p, params, MLP_NPARAM * 4, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_zero2, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, s.m, s.v, MLP_NPARAM);
  hipLaunchKernelGGL(k_mlp_quantise, dim3((MLP_HIDDEN * MLP_HIDDEN + 255) / 256), dim3(256), 0, st, s.p, s.W1, s.W2,
                     s.W2t);
  return hipGetLastError();
}

hipError_t mlp_get_params(const void* state, int rows, float* params, hipStream_t st) {
  const state_view s = carve(const_cast<void*>(state), rows);
  return hipMemcpyAsync(params, s.p, MLP_NPARAM * 4, hipMemcpyDeviceToDevice, st);
}

// Checkpoint of the training state: master weights and both Adam moments,
// [3][MLP_NPARAM] FP32.  Loading restores them and the bf16 copies.
hipError_t mlp_save_state(const void* state, int rows, float* out, hipStream_t st) {
  const state_view s = carve(const_cast<void*>(state), rows);
  const float* src[3] = {s.p, s.m, s.v};
  for (int i = 0; i < 3; ++i) {
    const hipError_t e = hipMemcpyAsync(out + (size_t)i * MLP_NPARAM, src[i], MLP_NPARAM * 4,
                                        hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t mlp_load_state(void* state, int rows, const float* in, hipStream_t st) {
  const state_view s = carve(state, rows);
  float* dst[3] = {s.p, s.m, s.v};
  for (int i = 0; i < 3; ++i) {
    const hipError_t e = hipMemcpyAsync(dst[i], in + (size_t)i * MLP_NPARAM, MLP_NPARAM * 4,
                                        hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_mlp_quantise, dim3((MLP_HIDDEN * MLP_HIDDEN + 255) / 256), dim3(256), 0, st, s.p, s.W1, s.W2,
                     s.W2t);
  return hipGetLastError();
}

// Forward, loss and backward over n <= rows rows: the gradient of the mean
// loss into the state (and into grads when not NULL), the loss into *loss.
hipError_t mlp_gradients(void* state, int rows, const float* X, const float* T, int n, float* loss, float* grads,
                         hipStream_t st) {
  const state_view s = carve(state, rows);
  const int nb = (n + RB - 1) / RB, nc = (n + 255) / 256;
  fwd_args a = {X, n, s.W1, s.W2, s.p + MLP_OFF_W3, s.p + MLP_OFF_B1, s.p + MLP_OFF_B2, s.p + MLP_OFF_B3,
                s.out, s.H1, s.H2};
  hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, st, s.out, T, n, s.p + MLP_OFF_W3, s.H2, s.dZ2, s.part);
  // loss / n, dW3, db3 from the per-block partials (in block order)
  const int hs = 2 + 2 * MLP_HIDDEN + 1;
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(256), 0, st, s.part, nb, 1, hs, loss);
  hipLaunchKernelGGL(k_mlp_scale, dim3(1), dim3(1), 0, st, loss, 1.0f / (float)n);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(256), 0, st, s.part + 1, nb, MLP_OUT * MLP_HIDDEN, hs,
                     s.g + MLP_OFF_W3);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(256), 0, st, s.part + 1 + MLP_OUT * MLP_HIDDEN, nb, MLP_OUT, hs,
                     s.g + MLP_OFF_B3);
  // dW2 = dZ2^T H1 and db2
  wgrad_args g2 = {s.dZ2, nullptr, MLP_HIDDEN, s.H1, nullptr, MLP_HIDDEN, n, s.part};
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(16, nc), dim3(64), 0, st, g2);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(MLP_HIDDEN * MLP_HIDDEN / 256), dim3(256), 0, st, s.part, nc,
                     MLP_HIDDEN * MLP_HIDDEN, MLP_HIDDEN * MLP_HIDDEN, s.g + MLP_OFF_W2);
  hipLaunchKernelGGL(k_mlp_bgrad, dim3(nc), dim3(MLP_HIDDEN), 0, st, s.dZ2, MLP_HIDDEN, n, s.part);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(MLP_HIDDEN), 0, st, s.part, nc, MLP_HIDDEN, MLP_HIDDEN,
                     s.g + MLP_OFF_B2);
  // dZ1 = (dZ2 W2) * [H1 > 0]; dW1 = dZ1^T X and db1
  hipLaunchKernelGGL(k_mlp_back_h1, dim3(nb), dim3(256), 0, st, s.dZ2, s.W2t, s.H1, n, s.dZ1);
  wgrad_args g1 = {s.dZ1, nullptr, MLP_HIDDEN, nullptr, X, MLP_FEAT, n, s.part};
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(4, nc), dim3(64), 0, st, g1);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(MLP_HIDDEN * MLP_FEAT / 256), dim3(256), 0, st, s.part, nc,
                     MLP_HIDDEN * MLP_FEAT, MLP_HIDDEN * MLP_FEAT, s.g + MLP_OFF_W1);
  hipLaunchKernelGGL(k_mlp_bgrad, dim3(nc), dim3(MLP_HIDDEN), 0, st, s.dZ1, MLP_HIDDEN, n, s.part);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(MLP_HIDDEN), 0, st, s.part, nc, MLP_HIDDEN, MLP_HIDDEN,
                     s.g + MLP_OFF_B1);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && grads) e = hipMemcpyAsync(grads, s.g, MLP_NPARAM * 4, hipMemcpyDeviceToDevice, st);
  return e;
}

// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the gradient in the
// state, then the bf16 copies.  step counts from 1.
hipError_t mlp_adam_step(void* state, int rows, float lr, int step, hipStream_t st) {
  const state_view s = carve(state, rows);
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f / (1.0f - powf(b1, (float)step)), c2 = 1.0f / (1.0f - powf(b2, (float)step));
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, s.p, s.m, s.v, s.g, MLP_NPARAM,
                     lr, b1, b2, 1e-8f, c1, c2);
  hipLaunchKernelGGL(k_mlp_quantise, dim3((MLP_HIDDEN * MLP_HIDDEN + 255) / 256), dim3(256), 0, st, s.p, s.W1, s.W2,
                     s.W2t);
  return hipGetLastError();
}

hipError_t mlp_export(const void* state, int rows, void* blob, hipStream_t st) {
  const state_view s = carve(const_cast<void*>(state), rows);
  hipLaunchKernelGGL(k_mlp_export, dim3((MLP_HIDDEN * MLP_HIDDEN + 255) / 256), dim3(256), 0, st, s.p,
                     (mlp_blob*)blob);
  return hipGetLastError();
}

}  // namespace cbp
