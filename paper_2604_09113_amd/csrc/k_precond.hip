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
// three dependent triangular solves.
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

template <typename T, int P, int NCE>
__global__ __launch_bounds__(256) void k_precond(const double* __restrict__ Sg, const double* __restrict__ cons,
                                                 const double* __restrict__ diagK, const double* __restrict__ Ktot,
                                                 const int* __restrict__ RU, int nx, T* __restrict__ Pout,
                                                 T* __restrict__ Psiout, double* __restrict__ Dout,
                                                 double* __restrict__ ScOut, int* __restrict__ flags) {
  constexpr int NU = 8 * P, NE = NU - 8, NCC = 4 * NCE, NC = 8 + NCC, NR = NE + NCC;
  constexpr int NSP = NU * (NU + 1) / 2;
  const int cell = blockIdx.x, tid = threadIdx.x;
  const bool left = (cell % nx) == 0;
  __shared__ T Sh[NE][NE + 1];
  __shared__ T Z[NE][NR + 1];
  __shared__ T Ch[NCC][NE];
  __shared__ T Cc[NCC][8];
  __shared__ T Tm[NCC][NCC];
  __shared__ T W2[NE][NCC];
  __shared__ T Scol[NE][8];
  __shared__ double Dv[NU];
  __shared__ double SPsi[NU * NC];
  __shared__ int bad;
  const double* S = Sg + (size_t)cell * NSP;
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < NE * NE; idx += 256) {
    int i = idx / NE, j = idx % NE, I = 8 + i, J = 8 + j;
    int hi = I > J ? I : J, lo = I > J ? J : I;
    Sh[i][j] = (T)S[hi * (hi + 1) / 2 + lo];
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
  // Cholesky of Shat (right-looking, unscaled trailing update, one barrier per column)
  for (int k = 0; k < NE; ++k) {
    const T akk = Sh[k][k];
    if (tid == 0 && !(akk > (T)0)) bad = 1;
    const T inv = (T)1 / akk;
    for (int idx = tid; idx < NE * NE; idx += 256) {
      int i = idx / NE, j = idx % NE;
      if (j > k && i >= j) Sh[i][j] -= Sh[i][k] * Sh[j][k] * inv;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < NE * NE; idx += 256) {
    int i = idx / NE, k = idx % NE;
    if (i > k) Sh[i][k] = Sh[i][k] / sqrt(Sh[k][k]);
  }
  __syncthreads();
  if (tid < NE) Sh[tid][tid] = sqrt(Sh[tid][tid]);
  // right-hand sides [I | Chat^T]
  for (int idx = tid; idx < NE * NR; idx += 256) {
    int i = idx / NR, j = idx % NR;
    Z[i][j] = j < NE ? (T)(i == j ? 1 : 0) : Ch[j - NE][i];
  }
  __syncthreads();
  // one thread per right-hand side: forward and backward substitution
  if (tid < NR) {
    const int j = tid;
    for (int k = 0; k < NE; ++k) {
      T zk = Z[k][j] / Sh[k][k];
      Z[k][j] = zk;
      for (int i = k + 1; i < NE; ++i) Z[i][j] -= Sh[i][k] * zk;
    }
    for (int k = NE - 1; k >= 0; --k) {
      T zk = Z[k][j];
      for (int i = k + 1; i < NE; ++i) zk -= Sh[i][k] * Z[i][j];
      Z[k][j] = zk / Sh[k][k];
    }
  }
  __syncthreads();
  // That = Chat X, masked rows get a unit diagonal (they carry no constraint)
  for (int idx = tid; idx < NCC * NCC; idx += 256) {
    int a = idx / NCC, b = idx % NCC;
    T s = 0;
    for (int i = 0; i < NE; ++i) s += Ch[a][i] * Z[i][NE + b];
    if (left && a == b && a < NCE) s = (T)1;
    Tm[a][b] = s;
  }
  __syncthreads();
  if (tid == 0) {  // small dense Cholesky of That
    for (int k = 0; k < NCC; ++k) {
      T d = Tm[k][k];
      for (int l = 0; l < k; ++l) d -= Tm[k][l] * Tm[k][l];
      if (!(d > (T)0)) { bad = 1; d = (T)1; }
      d = sqrt(d);
      Tm[k][k] = d;
      for (int i = k + 1; i < NCC; ++i) {
        T s = Tm[i][k];
        for (int l = 0; l < k; ++l) s -= Tm[i][l] * Tm[k][l];
        Tm[i][k] = s / d;
      }
    }
  }
  __syncthreads();
  // W2 = X That^-1 (row i solves That w = X[i,:]^T)
  if (tid < NE) {
    const int i = tid;
    T w[NCC];
    for (int a = 0; a < NCC; ++a) {
      T s = Z[i][NE + a];
      for (int l = 0; l < a; ++l) s -= Tm[a][l] * w[l];
      w[a] = s / Tm[a][a];
    }
    for (int a = NCC - 1; a >= 0; --a) {
      T s = w[a];
      for (int l = a + 1; l < NCC; ++l) s -= Tm[l][a] * w[l];
      w[a] = s / Tm[a][a];
    }
    for (int a = 0; a < NCC; ++a) W2[i][a] = w[a];
  }
  __syncthreads();
  // P = Shat^-1 - W2 X^T (in place in the first NE columns of Z)
  for (int idx = tid; idx < NE * NE; idx += 256) {
    int i = idx / NE, j = idx % NE;
    T s = Z[i][j];
    for (int a = 0; a < NCC; ++a) s -= W2[i][a] * Z[j][NE + a];
    Sh[i][j] = s;  // Sh is free after the solves; hold P there
  }
  __syncthreads();
  // store D_E P D_E packed lower
  T* Pc = Pout + (size_t)cell * (NE * (NE + 1) / 2);
  for (int idx = tid; idx < NE * (NE + 1) / 2; idx += 256) {
    int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= idx) ++i;
    while (i * (i + 1) / 2 > idx) --i;
    int j = idx - i * (i + 1) / 2;
    Pc[idx] = (T)(Dv[8 + i] * (double)Sh[i][j] * Dv[8 + j]);
  }
  // coarse basis Psi (NU x NC), kept in Z[0..NU) rows? Z has NE rows: store edge part in Z, corners implicit
  __syncthreads();
  for (int idx = tid; idx < NE * NC; idx += 256) {
    int i = idx / NC, j = idx % NC;
    T v;
    if (j < 8) {
      T s = 0;
      for (int k = 0; k < NE; ++k) s -= Sh[i][k] * Scol[k][j];
      for (int a = 0; a < NCC; ++a) s -= W2[i][a] * Cc[a][j];
      v = s;
    } else {
      v = W2[i][j - 8];
    }
    bool masked = left && (j == 0 || j == 1 || j == 4 || j == 5 || (j >= 8 && j < 8 + NCE));
    Z[i][j] = masked ? (T)0 : v;
  }
  __syncthreads();
  T* Pso = Psiout + (size_t)cell * NU * NC;
  for (int idx = tid; idx < NU * NC; idx += 256) {
    int i = idx / NC, j = idx % NC;
    double v;
    if (i < 8) {
      bool masked = left && (j == 0 || j == 1 || j == 4 || j == 5);
      v = (i == j && !masked) ? 1.0 : 0.0;
    } else {
      v = (double)Z[i - 8][j];
    }
    Pso[idx] = (T)(Dv[i] * v);
  }
  for (int j = tid; j < NU; j += 256) Dout[(size_t)cell * NU + j] = Dv[j];
  // S Psi in FP64 into W2-sized scratch: reuse Sh (P no longer needed)
  __syncthreads();
  for (int idx = tid; idx < NU * NC; idx += 256) {
    int i = idx / NC, j = idx % NC;
    double s = 0.0;
    for (int k = 0; k < NU; ++k) {
      int hi = i > k ? i : k, lo = i > k ? k : i;
      double psi;
      if (k < 8) {
        bool masked = left && (j == 0 || j == 1 || j == 4 || j == 5);
        psi = (k == j && !masked) ? 1.0 : 0.0;
      } else {
        psi = (double)Z[k - 8][j];
      }
      s += S[hi * (hi + 1) / 2 + lo] * psi;
    }
    SPsi[idx] = s;
  }
  __syncthreads();
  double* Sc = ScOut + (size_t)cell * (NC * (NC + 1) / 2);
  for (int idx = tid; idx < NC * NC; idx += 256) {
    int a = idx / NC, b = idx % NC;
    if (b > a) continue;
    double s = 0.0;
    for (int k = 0; k < NU; ++k) {
      double psi;
      if (k < 8) {
        bool masked = left && (a == 0 || a == 1 || a == 4 || a == 5);
        psi = (k == a && !masked) ? 1.0 : 0.0;
      } else {
        psi = (double)Z[k - 8][a];
      }
      s += psi * SPsi[k * NC + b];
    }
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
