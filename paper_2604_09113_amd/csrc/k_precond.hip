// Preconditioner setup per cell (A5-A7, Sec. 3.3 and Alg. 2).
//
// With the corner (cross-point) dofs removed (Alg. 2 step 3), the local saddle
// problem [S C^T; C 0] splits into the edge block Shat = S[E,E] and the edge
// constraints Chat.  Alg. 2 computes X = Shat^-1 Chat^T and That = Chat X
// (step 4) and, for a right-hand side fhat with zero prescribed coarse values,
// xhat = Shat^-1 fhat - X That^-1 X^T fhat.  That map is linear and fixed, so it
// is formed once here as the explicit symmetric fine operator
//   P = Shat^-1 - X That^-1 X^T,
// stored D-scaled (D_E P D_E) so that each PCG iteration applies the fine
// correction of Alg. 1 as one packed symmetric matrix-vector product instead of
// three dependent triangular solves.  Shat^-1 and That^-1 are formed by in-place
// Gauss-Jordan sweeps (both are SPD: no pivoting), whose pivot steps update
// every entry in parallel; the other steps are small matrix products.
//
// The coarse basis (Eq. of the local coarse problems) solves the same saddle
// problem with right-hand side [0; e_j].  For an edge constraint j that is
// xhat = X That^-1 e_j.  For a corner value j the prescribed unit value is
// moved to the right-hand side before removing the corner rows:
// fhat = -S[E, j], ghat = -C[edges, j], xhat = P fhat + X That^-1 ghat.
// The local coarse matrix is Psi^T S Psi (accumulated in FP64).
//
// Partition-of-unity weights (Sec. 3.3.3): D_jj = K_jj / sum over the cells
// sharing the dof of their K_jj.
//
// T = double (plain path) or float (mixed path: Shat, That, P, Psi in FP32).
#include "internal.h"

namespace lbddc {

// In-place Gauss-Jordan inverse of the SPD n x n block A (row stride LDA) by
// the 256 threads of the workgroup: rows go to the waves, columns to the lanes
// (n <= 64); colp is a length-n scratch.  Sets *bad on a non-positive pivot.
template <typename T, int LDA>
__device__ void gj_inverse(T* A, int n, T* colp, int* bad) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int l = 0; l < n; ++l) {
    if (threadIdx.x < n) colp[threadIdx.x] = A[threadIdx.x * LDA + l];
    __syncthreads();
    T piv = colp[l];
    if (!(piv > (T)0)) { if (threadIdx.x == 0) *bad = 1; piv = (T)1; }
    const T pinv = (T)1 / piv;
    const T rl = lane < n ? A[l * LDA + lane] : (T)0;  // pivot row, read before any write below
    __syncthreads();
    for (int i = wave; i < n; i += 4) {
      if (lane >= n) continue;
      T* a = A + i * LDA + lane;
      if (i == l) {
        *a = lane == l ? pinv : rl * pinv;
      } else {
        const T ci = colp[i] * pinv;
        *a = lane == l ? -ci : *a - ci * rl;
      }
    }
    __syncthreads();
  }
}

template <typename T, int P, int NCE>
__global__ __launch_bounds__(256) void k_precond(const double* __restrict__ Sg, const double* __restrict__ cons,
                                                 const double* __restrict__ diagK, const double* __restrict__ Ktot,
                                                 const int* __restrict__ RU, int nx, T* __restrict__ Pout,
                                                 T* __restrict__ Psiout, double* __restrict__ Dout,
                                                 double* __restrict__ ScOut, int* __restrict__ flags) {
  constexpr int NU = 8 * P, NE = NU - 8, NCC = 4 * NCE, NC = 8 + NCC;
  constexpr int NSP = NU * (NU + 1) / 2;
  static_assert(NU <= 64, "one row per lane");
  const int cell = blockIdx.x, tid = threadIdx.x;
  const bool left = (cell % nx) == 0;
  __shared__ T A[NE][NE + 1];     // Shat, then Shat^-1, then P
  __shared__ T X[NE][NCC + 1];    // Shat^-1 Chat^T
  __shared__ T W2[NE][NCC + 1];   // X That^-1
  __shared__ T Ch[NCC][NE];
  __shared__ T Cc[NCC][8];
  __shared__ T Tm[NCC][NCC + 1];  // That, then That^-1
  __shared__ T Scol[NE][8];
  __shared__ T colp[NE];
  __shared__ double Dv[NU];
  __shared__ double Ps[NU][NC + 1];   // coarse basis (unscaled)
  __shared__ double SPs[NU][NC + 1];  // S Psi
  __shared__ int bad;
  const double* S = Sg + (size_t)cell * NSP;
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < NE * NE; idx += 256) {
    int i = idx / NE, j = idx % NE, I = 8 + i, J = 8 + j;
    int hi = I > J ? I : J, lo = I > J ? J : I;
    A[i][j] = (T)S[hi * (hi + 1) / 2 + lo];
  }
  for (int idx = tid; idx < NE * 8; idx += 256) {
    int i = idx / 8, j = idx % 8, I = 8 + i;
    Scol[i][j] = (T)S[I * (I + 1) / 2 + j];
  }
  for (int j = tid; j < NU; j += 256) {
    int g = RU[(size_t)cell * NU + j];
    Dv[j] = g >= 0 ? diagK[(size_t)cell * NU + j] / Ktot[g] : 0.0;
  }
  // constraint rows: Chat (edge dofs) and the corner columns
  for (int idx = tid; idx < NCC * NE; idx += 256) Ch[idx / NE][idx % NE] = (T)0;
  for (int idx = tid; idx < NCC * 8; idx += 256) Cc[idx / 8][idx % 8] = (T)0;
  __syncthreads();
  const double* cc = cons + (size_t)cell * 4 * NCE * (P + 1) * 2;
  for (int idx = tid; idx < 4 * NCE * (P + 1) * 2; idx += 256) {
    const int comp = idx & 1, n = (idx >> 1) % (P + 1), et = (idx >> 1) / (P + 1);
    const int e = et / NCE;
    if (left && e == 0) continue;  // the clamped side carries no constraints
    const T v = (T)cc[idx];
    if (n == 0 || n == P) {
      int corner = (e == 0) ? (n == 0 ? 0 : 2) : (e == 1) ? (n == 0 ? 1 : 3) : (e == 2) ? (n == 0 ? 0 : 1) : (n == 0 ? 2 : 3);
      if (left && (corner == 0 || corner == 2)) continue;
      Cc[et][2 * corner + comp] = v;
    } else {
      Ch[et][2 * (e * (P - 1) + n - 1) + comp] = v;
    }
  }
  __syncthreads();
  // Shat^-1 in place
  gj_inverse<T, NE + 1>(&A[0][0], NE, colp, &bad);
  // X = Shat^-1 Chat^T
  for (int idx = tid; idx < NE * NCC; idx += 256) {
    const int i = idx / NCC, a = idx % NCC;
    T s = 0;
    for (int k = 0; k < NE; ++k) s += A[i][k] * Ch[a][k];
    X[i][a] = s;
  }
  __syncthreads();
  // That = Chat X; the clamped edge's rows carry no constraint and get a unit diagonal
  for (int idx = tid; idx < NCC * NCC; idx += 256) {
    const int a = idx / NCC, b = idx % NCC;
    T s = 0;
    for (int i = 0; i < NE; ++i) s += Ch[a][i] * X[i][b];
    if (left && a == b && a < NCE) s = (T)1;
    Tm[a][b] = s;
  }
  __syncthreads();
  gj_inverse<T, NCC + 1>(&Tm[0][0], NCC, colp, &bad);
  // W2 = X That^-1
  for (int idx = tid; idx < NE * NCC; idx += 256) {
    const int i = idx / NCC, a = idx % NCC;
    T s = 0;
    for (int b = 0; b < NCC; ++b) s += X[i][b] * Tm[b][a];
    W2[i][a] = s;
  }
  __syncthreads();
  // P = Shat^-1 - W2 X^T (in place)
  for (int idx = tid; idx < NE * NE; idx += 256) {
    const int i = idx / NE, j = idx % NE;
    T s = A[i][j];
    for (int a = 0; a < NCC; ++a) s -= W2[i][a] * X[j][a];
    A[i][j] = s;
  }
  __syncthreads();
  // store D_E P D_E packed lower
  T* Pc = Pout + (size_t)cell * (NE * (NE + 1) / 2);
  for (int i = tid >> 6; i < NE; i += 4)
    for (int j = tid & 63; j <= i; j += 64)
      Pc[i * (i + 1) / 2 + j] = (T)(Dv[8 + i] * (double)A[i][j] * Dv[8 + j]);
  // coarse basis Psi [NU][NC]: corner rows are the identity (masked on the
  // clamped side); edge rows: corner columns -P S[E, c] - W2 C[:, c], edge
  // constraint columns W2
  for (int idx = tid; idx < NU * NC; idx += 256) {
    const int i = idx / NC, j = idx % NC;
    const bool cmask = left && (j == 0 || j == 1 || j == 4 || j == 5);
    double v;
    if (i < 8) {
      v = (i == j && !cmask) ? 1.0 : 0.0;
    } else if (j < 8) {
      T s = 0;
      for (int k2 = 0; k2 < NE; ++k2) s -= A[i - 8][k2] * Scol[k2][j];
      for (int a = 0; a < NCC; ++a) s -= W2[i - 8][a] * Cc[a][j];
      v = cmask ? 0.0 : (double)s;
    } else {
      const bool emask = left && j < 8 + NCE;
      v = emask ? 0.0 : (double)W2[i - 8][j - 8];
    }
    Ps[i][j] = v;
  }
  __syncthreads();
  T* Pso = Psiout + (size_t)cell * NU * NC;
  for (int idx = tid; idx < NU * NC; idx += 256) {
    const int i = idx / NC, j = idx % NC;
    Pso[idx] = (T)(Dv[i] * Ps[i][j]);
  }
  for (int j = tid; j < NU; j += 256) Dout[(size_t)cell * NU + j] = Dv[j];
  // S Psi in FP64 (S packed lower, read through the cache), then Psi^T S Psi
  for (int idx = tid; idx < NU * NC; idx += 256) {
    const int i = idx / NC, j = idx % NC;
    const int ri = i * (i + 1) / 2;
    double s = 0.0;
    for (int k2 = 0; k2 <= i; ++k2) s += S[ri + k2] * Ps[k2][j];
    for (int k2 = i + 1; k2 < NU; ++k2) s += S[k2 * (k2 + 1) / 2 + i] * Ps[k2][j];
    SPs[i][j] = s;
  }
  __syncthreads();
  double* Sc = ScOut + (size_t)cell * (NC * (NC + 1) / 2);
  for (int idx = tid; idx < NC * NC; idx += 256) {
    const int a = idx / NC, b = idx % NC;
    if (b > a) continue;
    double s = 0.0;
    for (int k2 = 0; k2 < NU; ++k2) s += Ps[k2][a] * SPs[k2][b];
    Sc[a * (a + 1) / 2 + b] = s;
  }
  if (tid == 0 && bad) atomicOr(flags, 16);
}

// out[g] = sum over the owners of g of part[owner] (owners in fixed order)
__global__ void k_gather_sum(const double* __restrict__ part, const int* __restrict__ ptr,
                             const int* __restrict__ own, double* __restrict__ out, int N) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double s = 0.0;
  for (int o = ptr[g]; o < ptr[g + 1]; ++o) s += part[own[o]];
  out[g] = s;
}

hipError_t launch_weights(Ctx* c) {
  hipLaunchKernelGGL(k_gather_sum, dim3((c->NU + 255) / 256), dim3(256), 0, c->stream, c->d_diagK, c->d_uown_ptr,
                     c->d_uown, c->d_Ktot, c->NU);
  return hipGetLastError();
}

template <typename T>
static hipError_t precond_T(Ctx* c) {
  dim3 grid(c->ncell), block(256);
  T* Pout = (T*)c->d_P;
  T* Psi = (T*)c->d_Psi;
#define PC_CASE(pp, ncv)                                                                                          \
  if (c->p == pp && c->nce == ncv) {                                                                             \
    hipLaunchKernelGGL((k_precond<T, pp, ncv>), grid, block, 0, c->stream, c->d_S, c->d_cons, c->d_diagK,         \
                       c->d_Ktot, c->d_RU, c->nx, Pout, Psi, c->d_D, c->d_ScLoc, c->d_flags);                    \
    return hipGetLastError();                                                                                    \
  }
  PC_CASE(2, 2) PC_CASE(2, 3) PC_CASE(3, 2) PC_CASE(3, 3) PC_CASE(4, 2) PC_CASE(4, 3) PC_CASE(5, 2) PC_CASE(5, 3)
  PC_CASE(6, 2) PC_CASE(6, 3) PC_CASE(7, 2) PC_CASE(7, 3) PC_CASE(8, 2) PC_CASE(8, 3)
#undef PC_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_precond(Ctx* c, bool fp32) { return fp32 ? precond_T<float>(c) : precond_T<double>(c); }

}  // namespace lbddc
