// Local Schur complement (A4, Sec. 3.2): S = K_UU - K_UI K_II^-1 K_IU.
//
// The cell matrix in the permuted dof order [interior | skeleton] is factored
// by a right-looking Cholesky that stops after the interior columns: the
// eliminated columns hold L_II (rows < nI) and L_UI = (L_II^-1 K_IU)^T (rows
// >= nI), and the trailing block becomes S.  K_II^-1 is never formed.
//
// One workgroup of 256 threads per cell.  The lower triangle is distributed
// 2-D cyclically over a 16 x 16 thread grid and kept in registers (thread
// (tr, tc) owns rows tr + 16a, columns tc + 16b, a >= b); each elimination step
// broadcasts the pivot column through LDS (double-buffered, one barrier per
// column).  Elimination is organised in phases of 16 columns so that the
// register indices of the still-active blocks are compile-time constants.
//
// Outputs per cell: S packed lower row-major [nU(nU+1)/2], L_II packed
// row by row [nI(nI+1)/2] (row k holds columns 0..k), Y = L_II^-1 K_IU stored
// column by column [nU][nI] (the layouts the recovery reads coalesced), and
// the skeleton diagonal of K (for the weights).
// Skeleton slots of Dirichlet nodes (slots without a global skeleton dof: the
// cell edges on clamped sides) are replaced by identity rows/columns (their
// Dirichlet values are zero).
#include "internal.h"

namespace lbddc {

// 1 / sqrt(p) for p > 0: the hardware estimate refined by two Newton steps,
// y <- y (3/2 - p y^2 / 2), three dependent operations each: a shorter chain
// than the correctly rounded square root and division it replaces on the
// pivot step's critical path (every thread waits for this value).
__device__ __forceinline__ double rsqrt_refined(double p) {
  double y = __builtin_amdgcn_rsq(p);
  const double h = 0.5 * p;
#pragma unroll
  for (int i = 0; i < 2; ++i) y = fma(y, fma(-h * y, y, 0.5), y);
  return y;
}

template <int P>
__global__ __launch_bounds__(256) void k_schur(const double* __restrict__ K, const int* __restrict__ RU,
                                               double* __restrict__ S, double* __restrict__ L,
                                               double* __restrict__ Y, double* __restrict__ diagK,
                                               int* __restrict__ flags) {
  constexpr int NN = (P + 1) * (P + 1);
  constexpr int NDOF = 2 * NN, NI = 2 * (P - 1) * (P - 1), NU = 8 * P;
  constexpr int NA = (NDOF + 15) / 16, NPH = (NI + 15) / 16;
  constexpr int NPAIR = NN * (NN + 1) / 2;
  constexpr int NSP = NU * (NU + 1) / 2;
  const int cell = blockIdx.x;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  __shared__ double colbuf[2][256];
  __shared__ double pv[2][2];
  __shared__ double sst[NSP];
  __shared__ int msk[NU];
  for (int i = tid; i < NU; i += 256) msk[i] = RU[(size_t)cell * NU + i] < 0;
  __syncthreads();
  const double* Kc = K + (size_t)cell * NPAIR * 4;
  // every load of the thread's entries first, from clamped positions (entries
  // outside the lower triangle read entry 0 and are replaced below), so the
  // 66 loads are in flight together
  double A[NA][NA];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int I = tr + 16 * a, J = tc + 16 * b;
      const bool in = I < NDOF && J <= I;
      const int Ic = in ? I : 0, Jc = in ? J : 0, n1 = Ic >> 1, n2 = Jc >> 1;
      A[a][b] = Kc[((size_t)(n1 * (n1 + 1) / 2 + n2)) * 4 + 2 * (Ic & 1) + (Jc & 1)];
    }
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int I = tr + 16 * a, J = tc + 16 * b;
      double v = 0.0;
      if (I < NDOF && J <= I) {
        v = A[a][b];
        const bool mI = I >= NI && msk[I - NI], mJ = J >= NI && msk[J - NI];
        if (I == J && I >= NI) diagK[(size_t)cell * NU + I - NI] = mI ? 0.0 : v;
        if (mI || mJ) v = (I == J) ? 1.0 : 0.0;
      }
      A[a][b] = v;
    }
  int buf = 0;
  bool bad = false;
  double* Lc = L + (size_t)cell * (NI * (NI + 1) / 2);
  double* Yc = Y + (size_t)cell * NI * NU;
  // colbuf[buf][I] = column k below the pivot (zero for I <= k and past NDOF),
  // pv[buf] = {pivot, 1/sqrt(pivot)}: the updates below then need no masks
  // (rows and columns at or above the pivot meet zeros; the eliminated
  // columns, already stored as L and Y, are not read again)
  for (int i = tid; i < 2 * 256; i += 256) (&colbuf[0][0])[i] = 0.0;
  __syncthreads();
#pragma unroll
  for (int ph = 0; ph < NPH; ++ph) {
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * ph + kk;
      if (k >= NI) break;
      if (tc == kk) {
#pragma unroll
        for (int a = ph; a < NA; ++a) {
          const int I = tr + 16 * a;
          if (I < NDOF) colbuf[buf][I] = I > k ? A[a][ph] : 0.0;
        }
        if (tr == kk) {
          double p0 = A[ph][ph];
          if (!(p0 > 0.0)) { bad = true; p0 = 1.0; }
          pv[buf][0] = p0;
          pv[buf][1] = rsqrt_refined(p0);
        }
      }
      __syncthreads();
      const double rinv = pv[buf][1];
      if (tid >= k && tid < NDOF) {
        if (tid < NI) Lc[tid * (tid + 1) / 2 + k] = tid == k ? sqrt(pv[buf][0]) : colbuf[buf][tid] * rinv;
        else Yc[(size_t)(tid - NI) * NI + k] = colbuf[buf][tid] * rinv;
      }
      double lr[NA], lcv[NA];
#pragma unroll
      for (int a = ph; a < NA; ++a) {
        lr[a] = colbuf[buf][tr + 16 * a] * rinv;
        lcv[a] = colbuf[buf][tc + 16 * a] * rinv;
      }
#pragma unroll
      for (int a = ph; a < NA; ++a)
#pragma unroll
        for (int b = ph; b <= a; ++b) A[a][b] -= lr[a] * lcv[b];
      buf ^= 1;
    }
  }
  if (bad) atomicOr(flags, 8);
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int I = tr + 16 * a, J = tc + 16 * b;
      if (I < NDOF && J >= NI && J <= I) {
        const int i = I - NI, j = J - NI;
        sst[i * (i + 1) / 2 + j] = A[a][b];
      }
    }
  __syncthreads();
  double* Sc = S + (size_t)cell * NSP;
  for (int i = tid; i < NSP; i += 256) Sc[i] = sst[i];
}

hipError_t launch_schur(Ctx* c) {
  dim3 grid(c->ncell), block(256);
#define SC_CASE(pp)                                                                                             \
  case pp:                                                                                                      \
    hipLaunchKernelGGL(k_schur<pp>, grid, block, 0, c->stream, c->d_K, c->d_RU, c->d_S, c->d_L, \
                       c->d_Y, c->d_diagK, c->d_flags);                                                        \
    break;
  switch (c->p) {
    SC_CASE(2) SC_CASE(3) SC_CASE(4) SC_CASE(5) SC_CASE(6) SC_CASE(7) SC_CASE(8) SC_CASE(9) SC_CASE(10)
    default: return hipErrorInvalidValue;
  }
#undef SC_CASE
  return hipGetLastError();
}

}  // namespace lbddc
