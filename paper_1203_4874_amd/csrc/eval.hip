// Unit-circle evaluation of the blurred frames (Sec. 4 eq. 3; Sec. 5: the
// evaluation at points around the unit circle is a DFT along one axis).
//
// For w_j = exp(-2 pi i j / S):
//   EX[j][x] = sum_y B[y][x] w_j^y = sum_{r<S} w_j^r F[r][x],  F[r][x] = sum_{y = r mod S} B[y][x]
//   EY[i][y] = sum_x B[y][x] w_i^x = sum_{r<S} w_i^r G[y][r],  G[y][r] = sum_{x = r mod S} B[y][x]
// i.e. a fold of the frame modulo S along one axis (one FP64 add per pixel)
// followed by an S-point DFT.  All accumulation is FP64 whatever the frame
// type.  The column fold runs over row groups and residues (partials per
// group, summed in a fixed order by the evaluation kernel), the row fold one
// row per wave.
//
// Layouts (cf = 2*channel + frame):
//   fpart [RG][ncf][S][Wmax] double, EX [ncf][S][Wmax] c64, EY [ncf][S][Hmax] c64.
// The row evaluation of a deblurring call is done by the forward row FFT
// kernel (same arithmetic, same order) from the rows it loads anyway;
// k_eval_rows serves kernel-only calls and the one-frame evaluation.
#include "eigsmall.h"
#include "internal.h"

namespace cbp {

namespace {

template <typename T>
__device__ inline void pick(const frame_desc& d, int cf, const T*& b, int64_t& pitch, int& H, int& W) {
  const int ch = cf >> 1;
  if ((cf & 1) == 0) { b = (const T*)d.b1 + ch * d.cs1; pitch = d.p1; H = d.H1; W = d.W1; }
  else { b = (const T*)d.b2 + ch * d.cs2; pitch = d.p2; H = d.H2; W = d.W2; }
}

// Column fold over rows [g*rpg, (g+1)*rpg) of one (channel, frame): one
// thread per (column, residue r), summing the rows y = r mod S of the group
// in increasing order (up to sixteen loads in flight), 64 columns per item.
// Items: (column block, residue, row group, cf).
// Twiddle tables exp(-2 pi i t / P) of the row and column FFTs (the row
// table also in FP64 for the kernel spectra); an item is 256 consecutive
// indices of [0, Px + Py), the row table first.  The FP64 value is rounded
// once to T, so an entry equals what an in-place evaluation would give.
template <typename T>
__device__ inline void twiddle_item(const frame_desc& d, int item) {
  for (int u = threadIdx.x; u < 256; u += blockDim.x) {
    const int t = item * 256 + u;
    if (t < d.Px) {
      double s, c;
      sincospi(-2.0 * (double)t / (double)d.Px, &s, &c);
      d.twxd[t] = {c, s};
    }
  }
}

// Workgroups [0, gf) fold; the rest fill the twiddle tables.  With an inline
// head (ih.ndesc_bytes > 0) every workgroup reads the descriptors and prefix
// sums from the launch's arguments and workgroup 0 stores them at br's place
// in the workspace head for the later launches.
template <typename T>
__global__ __launch_bounds__(64) void k_fold_cols(batch_ref br_ws, int gf, inline_head ih) {
  batch_ref br = br_ws;
  // the call's item counters start at zero (the later launches of the
  // chunk hand out their items from them)
  if (blockIdx.x == 0 && br_ws.ctr != nullptr)
    for (int i = threadIdx.x; i < CTR_COUNT; i += blockDim.x) br_ws.ctr[i] = 0;
  if (ih.ndesc_bytes > 0) {
    br.descs = (const frame_desc*)ih.bytes;
    br.starts = (const int*)(ih.bytes + ih.ndesc_bytes);
    if (blockIdx.x == 0) {
      const uint4* src = (const uint4*)ih.bytes;
      uint4* dd = (uint4*)br_ws.descs;
      uint4* ds = (uint4*)br_ws.starts;
      const int nd = ih.ndesc_bytes / 16, ns = ih.nstart_bytes / 16;
      for (int i = threadIdx.x; i < nd; i += blockDim.x) dd[i] = src[i];
      for (int i = threadIdx.x; i < ns; i += blockDim.x) ds[i] = src[nd + i];
    }
  }
  if ((int)blockIdx.x >= gf) {
    for_items_part<Q_TWID>(br, (int)blockIdx.x - gf, (int)gridDim.x - gf,
                           [&](const frame_desc& d, int item) __attribute__((always_inline)) {
                             twiddle_item<T>(d, item);
                           });
    return;
  }
  for_items_part<Q_FOLD>(br, (int)blockIdx.x, gf, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int S = d.S;
    const int nx = (d.Wmax + 63) / 64;
    const int bx = item % nx;
    int rest = item / nx;
    const int r = rest % S;
    rest /= S;
    const int g = rest % d.RG, cf = rest / d.RG;
    const T* b;
    int64_t pitch;
    int H, W;
    pick(d, cf, b, pitch, H, W);
    const int x = bx * 64 + threadIdx.x;
    if (x >= W) return;
    const int y1 = min(g * d.rpg + d.rpg, H);
    const T* col = b + x;
    double acc = 0.0;
    int y = g * d.rpg + r;
    // sixteen loads in flight, then added in increasing y
    for (; y + 15 * S < y1; y += 16 * S) {
      T v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = col[(int64_t)(y + u * S) * pitch];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += (double)v[u];
    }
    for (; y + 3 * S < y1; y += 4 * S) {
      const T v0 = col[(int64_t)y * pitch], v1 = col[(int64_t)(y + S) * pitch];
      const T v2 = col[(int64_t)(y + 2 * S) * pitch], v3 = col[(int64_t)(y + 3 * S) * pitch];
      acc += (double)v0;
      acc += (double)v1;
      acc += (double)v2;
      acc += (double)v3;
    }
    for (; y < y1; y += S) acc += (double)col[(int64_t)y * pitch];
    d.fpart[(((size_t)g * d.ncf + cf) * S + r) * (size_t)d.Wmax + x] = acc;
  });
}

// The column evaluation on its own (kernel-only calls; a deblurring call runs
// it on extra workgroups of the row-pass launch).  Items: (column block, cf).
__global__ __launch_bounds__(256) void k_eval_cols(batch_ref br) {
  __shared__ double F[CBP_MAX_S][16];
  __shared__ c64 tw[CBP_MAX_S];
  for_items<Q_EVAL_COLS>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    eval_cols_item(d, item, F, tw);
  });
}

// Row fold and S-point DFT: two waves per row.  With G = floor(128 / S)
// lane groups, lane l = g S + r (g < G) of the pair sums the row entries
// x = r + S (g + G i), i = 0, 1, ... in order; residue r is then the sum of
// its G partials in group order.  k_row_fwd folds the rows it holds with the
// same lanes and the same order, so both give the same bits.
// Items: (pair of rows, cf).
template <typename T>
__global__ __launch_bounds__(256) void k_eval_rows(batch_ref br) {
  __shared__ double part[2][128];
  __shared__ double g[2][CBP_MAX_S];
  __shared__ c64 tw[CBP_MAX_S];
  for_items<Q_EVAL_ROWS>(br, [&](const frame_desc& d, int item) __attribute__((always_inline)) {
    const int ny = (d.Hmax + 1) / 2;
    const int by = item % ny, cf = item / ny;
    const int S = d.S, G = 128 / S;
    const T* b;
    int64_t pitch;
    int H, W;
    pick(d, cf, b, pitch, H, W);
    const int w = threadIdx.x >> 7, l = threadIdx.x & 127;
    const int y = by * 2 + w;
    const int gl = l / S, r = l - gl * S;
    unit_twiddles(tw, S);
    double acc = 0.0;
    if (y < H && gl < G) acc = fold_strided(b + (int64_t)y * pitch, 1, r + S * gl, S * G, W);
    part[w][l] = acc;
    __syncthreads();
    if (l < S) {
      double sr = part[w][l];
      for (int q = 1; q < G; ++q) sr += part[w][q * S + l];
      g[w][l] = sr;
    }
    __syncthreads();
    if (y < H && l < S) d.ey[((size_t)cf * S + l) * d.Hmax + y] = dft_at(g[w], 1, tw, S, l);
  });
}

}  // namespace

template <typename T>
hipError_t launch_fold(const batch_ref& br, int grid, int twid_grid, const inline_head* ih, hipStream_t st) {
  prof_begin(PH_FOLD, st);
  inline_head h;
  if (ih) h = *ih;
  else h.ndesc_bytes = h.nstart_bytes = 0;
  hipLaunchKernelGGL(k_fold_cols<T>, dim3(grid + twid_grid), dim3(64), 0, st, br, grid, h);
  prof_end(PH_FOLD, st);
  return hipGetLastError();
}

hipError_t launch_eval_cols(const batch_ref& br, int grid, hipStream_t st) {
  prof_begin(PH_EVAL_COLS, st);
  hipLaunchKernelGGL(k_eval_cols, dim3(grid), dim3(256), 0, st, br);
  prof_end(PH_EVAL_COLS, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_eval_rows(const batch_ref& br, int grid, hipStream_t st) {
  prof_begin(PH_EVAL_ROWS, st);
  hipLaunchKernelGGL(k_eval_rows<T>, dim3(grid), dim3(256), 0, st, br);
  prof_end(PH_EVAL_ROWS, st);
  return hipGetLastError();
}

template hipError_t launch_fold<float>(const batch_ref&, int, int, const inline_head*, hipStream_t);
template hipError_t launch_fold<double>(const batch_ref&, int, int, const inline_head*, hipStream_t);
template hipError_t launch_eval_rows<float>(const batch_ref&, int, hipStream_t);
template hipError_t launch_eval_rows<double>(const batch_ref&, int, hipStream_t);

}  // namespace cbp
