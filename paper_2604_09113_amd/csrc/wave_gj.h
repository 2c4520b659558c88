// Helpers shared by the preconditioner setup and the coarse factorisation: a
// refined reciprocal for pivots, a broadcast of one lane's value, and an
// in-register Gauss-Jordan inverse of a small SPD block by one wave.
#pragma once

#include <hip/hip_runtime.h>

namespace lbddc {

// 1 / p for a pivot p: the hardware reciprocal estimate refined by Newton
// steps y <- y + y (1 - p y) (two in FP64, one in FP32), a shorter dependent
// chain than the correctly rounded division on a pivot step's critical path.
__device__ __forceinline__ double recip_refined(double p) {
  double y = __builtin_amdgcn_rcp(p);
#pragma unroll
  for (int i = 0; i < 2; ++i) y = fma(y, fma(-p, y, 1.0), y);
  return y;
}
__device__ __forceinline__ float recip_refined(float p) {
  const float y = __builtin_amdgcn_rcpf(p);
  return fmaf(y, fmaf(-p, y, 1.0f), y);
}

// Value of v held by lane `src` (wave-uniform), through scalar reads.
__device__ __forceinline__ float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// In-place Gauss-Jordan inverse of the SPD N x N block A (row stride LDA,
// N <= 64; no pivoting) by wave 0 alone, with lane j holding column j in
// registers.  Pivot step l:
//   A[l][j] <- A[l][j] / p (1 / p on the diagonal),
//   A[i][j] <- A[i][j] - (A[i][l] / p) A[l][j], A[i][l] <- -A[i][l] / p  (i != l).
// The register array is rotated by one row per step, so that row l sits at
// index 0 at step l and every index is a compile-time constant (after N steps
// the rows are back in order); the pivot column entries A[i][l] come from lane
// l by readlane.  A step needs neither a barrier nor LDS traffic.  Sets *bad
// on a non-positive pivot.  The other waves wait at the closing barrier.
template <typename T, int LDA, int N>
__device__ __forceinline__ void gj_inverse_wave(T* A, int* bad) {
  static_assert(N <= 64, "one column per lane");
  if (threadIdx.x < 64) {
    // lanes j >= N carry a copy of column 0 through the sweep: their values
    // are never read by other lanes nor stored
    const int j = threadIdx.x, jc = j < N ? j : 0;
    T col[N];
#pragma unroll
    for (int i = 0; i < N; ++i) col[i] = A[i * LDA + jc];
    for (int l = 0; l < N; ++l) {
      const T rl = col[0];  // A[l][j]
      T piv = lane_bcast(rl, l);
      if (!(piv > (T)0)) {
        if (j == 0) *bad = 1;
        piv = (T)1;
      }
      const T pinv = recip_refined(piv);
      const bool jl = j == l;
#pragma unroll
      for (int i = 1; i < N; ++i) {
        const T ci = lane_bcast(col[i], l) * pinv;
        col[i - 1] = jl ? -ci : col[i] - ci * rl;
      }
      col[N - 1] = jl ? pinv : rl * pinv;
    }
    if (j < N) {
#pragma unroll
      for (int i = 0; i < N; ++i) A[i * LDA + j] = col[i];
    }
  }
  __syncthreads();
}

}  // namespace lbddc
