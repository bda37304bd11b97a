// Internal launch interface between the C ABI (api.hip) and the kernel
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

#include "cbp.h"
#include "common.h"
#include "fft_core.h"

namespace cbp {

// One blurred pair as the kernels see it (device pointers, element pitches).
template <typename T>
struct pair_view {
  const T* b1;
  const T* b2;
  int64_t p1, p2;    // row pitch (elements)
  int64_t cs1, cs2;  // channel stride (elements)
  int H1, W1, H2, W2;
  int nch;
};

// Geometry and workspace offsets of one frame (all offsets in bytes from the
// frame's workspace base).
struct frame_plan {
  int H1, W1, H2, W2, Hmax, Wmax;
  int m, n, k1, k2, S, N;  // N = k1 + k2
  int nch;
  int rpg, RG;             // fold row-group size (multiple of S) and count
  int Py, Px, hx;          // FFT grid and half-spectrum width
  int cw;                  // columns per workgroup in the column pass
  fft_plan fy, fx;
  size_t off_fpart, off_ex, off_ey, off_corr, off_xvec, off_lam0, off_pq, off_cbuf, off_kern,
      off_t1, off_t2, off_u, total;
};

// ---------------------------------------------------------------- phase timing
// Phases of one call, in launch order (also the names cbp_profile_phase_name
// returns).
enum phase_id {
  PH_FOLD = 0, PH_EVAL_COLS, PH_EVAL_ROWS, PH_GRAM, PH_SAMPLE, PH_FINALIZE,
  PH_ROW_FWD, PH_COL_FILTER, PH_ROW_INV, PH_COUNT
};
// Record the start / end of a phase on a stream when timing is enabled
// (no-ops otherwise).  Implemented in api.hip.
void prof_begin(int phase, hipStream_t st);
void prof_end(int phase, hipStream_t st);

// ---------------------------------------------------------------- launchers
// eval.hip
template <typename T>
hipError_t launch_eval_cols(const pair_view<T>& v, const frame_plan& fp, char* ws, hipStream_t st);
template <typename T>
hipError_t launch_eval_rows(const pair_view<T>& v, const frame_plan& fp, char* ws, hipStream_t st);
hipError_t launch_eval_single(const void* b, int dtype, int64_t pitch, int H, int W, int S,
                              char* ws, double* ex, double* ey, hipStream_t st);

// recover.hip
hipError_t launch_recover(const frame_plan& fp, char* ws, double* K1, double* K2, void* diag,
                          hipStream_t st);

// fft.hip
template <typename T>
hipError_t launch_row_fwd(const pair_view<T>& v, const frame_plan& fp, char* ws, hipStream_t st);
template <typename T>
hipError_t launch_col_inv(const pair_view<T>& v, const frame_plan& fp, char* ws, const double* K1,
                          const double* K2, T* out, int64_t opitch, int64_t ocs, double lambda,
                          hipStream_t st);

}  // namespace cbp
