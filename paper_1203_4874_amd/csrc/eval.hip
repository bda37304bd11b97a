// Unit-circle evaluation of the blurred frames (Sec. 4 eq. 3; Sec. 5: the
// evaluation at points around the unit circle is a DFT along one axis).
//
// For w_j = exp(-2 pi i j / S):
//   EX[j][x] = sum_y B[y][x] w_j^y = sum_{r<S} w_j^r F[r][x],  F[r][x] = sum_{y = r mod S} B[y][x]
//   EY[i][y] = sum_x B[y][x] w_i^x = sum_{r<S} w_i^r G[y][r],  G[y][r] = sum_{x = r mod S} B[y][x]
// i.e. a fold of the frame modulo S along one axis (one FP64 add per pixel)
// followed by an S-point DFT.  All accumulation is FP64 whatever the frame
// type.  The column fold runs over row groups (partials per group, summed in
// a fixed order by the evaluation kernel), the row fold one row per wave.
//
// Layouts (cf = 2*channel + frame):
//   fpart [RG][ncf][S][Wmax] double, EX [ncf][S][Wmax] c64, EY [ncf][S][Hmax] c64.
#include "eigsmall.h"
#include "internal.h"

namespace cbp {

namespace {

template <typename T>
__device__ inline void pick(const pair_view<T>& v, int cf, const T*& b, int64_t& pitch, int& H, int& W) {
  const int ch = cf >> 1;
  if ((cf & 1) == 0) { b = v.b1 + ch * v.cs1; pitch = v.p1; H = v.H1; W = v.W1; }
  else { b = v.b2 + ch * v.cs2; pitch = v.p2; H = v.H2; W = v.W2; }
}

__device__ inline void unit_twiddles(c64* tw, int S) {
  for (int t = threadIdx.x; t < S; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)S, &s, &c);
    tw[t] = {c, s};
  }
}

// Column fold over rows [g*rpg, (g+1)*rpg) of one (channel, frame): one
// thread per column, S independent accumulators, 64 columns per workgroup.
template <typename T>
__global__ __launch_bounds__(64) void k_fold_cols(pair_view<T> v, int S, int rpg, double* fpart, int Wmax) {
  const int cf = blockIdx.z, ncf = gridDim.z;
  const T* b;
  int64_t pitch;
  int H, W;
  pick(v, cf, b, pitch, H, W);
  const int x = blockIdx.x * 64 + threadIdx.x;
  if (x >= W) return;
  const int y0 = blockIdx.y * rpg;
  const int y1 = min(y0 + rpg, H);
  double acc[CBP_MAX_S];
#pragma unroll
  for (int r = 0; r < CBP_MAX_S; ++r) acc[r] = 0.0;
  for (int yb = y0; yb < y1; yb += S) {
    const T* col = b + (int64_t)yb * pitch + x;
#pragma unroll
    for (int r = 0; r < CBP_MAX_S; ++r)
      if (r < S && yb + r < y1) acc[r] += (double)col[(int64_t)r * pitch];
  }
  double* out = fpart + ((size_t)blockIdx.y * ncf + cf) * S * (size_t)Wmax + x;
#pragma unroll
  for (int r = 0; r < CBP_MAX_S; ++r)
    if (r < S) out[(size_t)r * Wmax] = acc[r];
}

// Sum the row-group partials of the column fold and apply the S-point DFT;
// 16 columns per workgroup, 16 residues / frequencies in flight per column.
__global__ __launch_bounds__(256) void k_eval_cols(const double* fpart, int RG, int S, int Wmax, int W1, int W2,
                                                   c64* ex, int exW) {
  __shared__ double F[CBP_MAX_S][16];
  __shared__ c64 tw[CBP_MAX_S];
  const int cf = blockIdx.y, ncf = gridDim.y;
  const int W = (cf & 1) ? W2 : W1;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int x = blockIdx.x * 16 + tx;
  unit_twiddles(tw, S);
  for (int r = ty; r < S; r += 16) {
    double s0 = 0.0, s1 = 0.0;
    if (x < W) {
      const double* p = fpart + ((size_t)cf * S + r) * Wmax + x;
      const size_t gs = (size_t)ncf * S * Wmax;
      int g = 0;
      for (; g + 2 <= RG; g += 2) {
        s0 += p[(size_t)g * gs];
        s1 += p[(size_t)(g + 1) * gs];
      }
      if (g < RG) s0 += p[(size_t)g * gs];
    }
    F[r][tx] = s0 + s1;
  }
  __syncthreads();
  if (x >= W) return;
  for (int j = ty; j < S; j += 16) {
    c64 acc = {0.0, 0.0};
    int t = 0;
    for (int r = 0; r < S; ++r) {
      const double f = F[r][tx];
      acc.re += f * tw[t].re;
      acc.im += f * tw[t].im;
      t += j;
      if (t >= S) t -= S;
    }
    ex[((size_t)cf * S + j) * exW + x] = acc;
  }
}

// Row fold and S-point DFT: one wave per row; lane l folds the chunks
// x in [q S, q S + S), q = l, l + 64, ...; wave shuffles sum the lanes.
template <typename T>
__global__ __launch_bounds__(256) void k_eval_rows(pair_view<T> v, int S, c64* ey, int eyH) {
  __shared__ double g[4][CBP_MAX_S];
  __shared__ c64 tw[CBP_MAX_S];
  const int cf = blockIdx.y;
  const T* b;
  int64_t pitch;
  int H, W;
  pick(v, cf, b, pitch, H, W);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int y = blockIdx.x * 4 + w;
  unit_twiddles(tw, S);
  double acc[CBP_MAX_S];
#pragma unroll
  for (int r = 0; r < CBP_MAX_S; ++r) acc[r] = 0.0;
  if (y < H) {
    const T* row = b + (int64_t)y * pitch;
    for (int x0 = l * S; x0 < W; x0 += 64 * S) {
#pragma unroll
      for (int r = 0; r < CBP_MAX_S; ++r)
        if (r < S && x0 + r < W) acc[r] += (double)row[x0 + r];
    }
  }
#pragma unroll
  for (int r = 0; r < CBP_MAX_S; ++r) {
    if (r < S) {
      const double s = wsum(acc[r]);
      if (l == 0) g[w][r] = s;
    }
  }
  __syncthreads();
  if (y < H && l < S) {
    c64 e = {0.0, 0.0};
    int t = 0;
    for (int r = 0; r < S; ++r) {
      const double f = g[w][r];
      e.re += f * tw[t].re;
      e.im += f * tw[t].im;
      t += l;
      if (t >= S) t -= S;
    }
    ey[((size_t)cf * S + l) * eyH + y] = e;
  }
}

}  // namespace

template <typename T>
hipError_t launch_eval_cols(const pair_view<T>& v, const frame_plan& fp, char* ws, hipStream_t st) {
  const int ncf = 2 * v.nch;
  double* fpart = (double*)(ws + fp.off_fpart);
  c64* ex = (c64*)(ws + fp.off_ex);
  const int S = fp.S;
  prof_begin(PH_FOLD, st);
  hipLaunchKernelGGL(k_fold_cols<T>, dim3((fp.Wmax + 63) / 64, fp.RG, ncf), dim3(64), 0, st, v, S, fp.rpg,
                     fpart, fp.Wmax);
  prof_end(PH_FOLD, st);
  prof_begin(PH_EVAL_COLS, st);
  hipLaunchKernelGGL(k_eval_cols, dim3((fp.Wmax + 15) / 16, ncf), dim3(256), 0, st, fpart, fp.RG, S, fp.Wmax,
                     v.W1, v.W2, ex, fp.Wmax);
  prof_end(PH_EVAL_COLS, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_eval_rows(const pair_view<T>& v, const frame_plan& fp, char* ws, hipStream_t st) {
  const int ncf = 2 * v.nch;
  c64* ey = (c64*)(ws + fp.off_ey);
  prof_begin(PH_EVAL_ROWS, st);
  hipLaunchKernelGGL(k_eval_rows<T>, dim3((fp.Hmax + 3) / 4, ncf), dim3(256), 0, st, v, fp.S, ey, fp.Hmax);
  prof_end(PH_EVAL_ROWS, st);
  return hipGetLastError();
}

template hipError_t launch_eval_cols<float>(const pair_view<float>&, const frame_plan&, char*, hipStream_t);
template hipError_t launch_eval_cols<double>(const pair_view<double>&, const frame_plan&, char*, hipStream_t);
template hipError_t launch_eval_rows<float>(const pair_view<float>&, const frame_plan&, char*, hipStream_t);
template hipError_t launch_eval_rows<double>(const pair_view<double>&, const frame_plan&, char*, hipStream_t);

// One frame, channel 0, written straight to the caller's EX (S x W) and EY (S x H).
hipError_t launch_eval_single(const void* b, int dtype, int64_t pitch, int H, int W, int S, char* ws, double* ex,
                              double* ey, hipStream_t st) {
  const int rpg = S * ((32 + S - 1) / S);
  const int RG = (H + rpg - 1) / rpg;
  double* fpart = (double*)ws;
  auto run = [&](auto* ptr) -> hipError_t {
    using T = typename std::remove_const<typename std::remove_pointer<decltype(ptr)>::type>::type;
    pair_view<T> v{ptr, ptr, pitch, pitch, 0, 0, H, W, H, W, 1};
    hipLaunchKernelGGL(k_fold_cols<T>, dim3((W + 63) / 64, RG, 1), dim3(64), 0, st, v, S, rpg, fpart, W);
    hipLaunchKernelGGL(k_eval_cols, dim3((W + 15) / 16, 1), dim3(256), 0, st, fpart, RG, S, W, W, W, (c64*)ex, W);
    hipLaunchKernelGGL(k_eval_rows<T>, dim3((H + 3) / 4, 1), dim3(256), 0, st, v, S, (c64*)ey, H);
    return hipGetLastError();
  };
  if (dtype == 0) return run((const float*)b);
  return run((const double*)b);
}

}  // namespace cbp
