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
// T is the arithmetic, TO the stored precision of P and Psi: double/double on
// the plain path; double/float on the mixed path, whose solve streams P and
// Psi in FP32.  Forming the inverses in FP64 keeps the stored operator within
// FP32 rounding of the FP64 one even when rho makes Shat ill conditioned (an
// FP32 Gauss-Jordan loses about cond(Shat) times FP32 epsilon).
#include "internal.h"
#include "wave_gj.h"

namespace lbddc {

typedef float flt4m __attribute__((ext_vector_type(4)));
typedef double dbl4m __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 in the precision T.  Operands: lane l gives A[m = l % 16][k = l / 16]
// and B[k = l / 16][n = l % 16]; value v of the result sits at column l % 16 and
// row row(l, v).
template <typename T> struct Mf;
template <> struct Mf<float> {
  typedef flt4m v4;
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <> struct Mf<double> {
  typedef dbl4m v4;
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};

// C = A B (M x N, depth K) on MFMA by the workgroup's four waves, one 16 x 16
// output tile per wave at a time (operands past M, N, K are zero):
// a(i, k) and b(k, j) read the operands, out(i, j, value) takes each result.
template <typename T, int M, int N, int K, typename FA, typename FB, typename FO>
__device__ __forceinline__ void mfma_mm(FA a, FB b, FO out) {
  typedef typename Mf<T>::v4 v4;
  constexpr int TM = (M + 15) / 16, TN = (N + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kl = lane >> 4;
  for (int t = wave; t < TM * TN; t += 4) {
    const int r0 = (t / TN) * 16, c0 = (t % TN) * 16;
    v4 acc = v4{0, 0, 0, 0};
    // bounds that hold for every tile are known at compile time, so operand
    // reads from memory need no branch (and no wait per read)
    const bool row_ok = M % 16 == 0 || r0 + l16 < M, col_ok = N % 16 == 0 || c0 + l16 < N;
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + kl;
      const bool k_ok = K % 4 == 0 || k < K;
      const T av = (row_ok && k_ok) ? a(r0 + l16, k) : (T)0;
      const T bv = (k_ok && col_ok) ? b(k, c0 + l16) : (T)0;
      acc = Mf<T>::op(av, bv, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = r0 + Mf<T>::row(lane, v), j = c0 + l16;
      if (i < M && j < N) out(i, j, acc[v]);
    }
  }
}

template <typename T, typename TO, int P, int NCE>
__global__ __launch_bounds__(256) void k_precond(const double* __restrict__ Sg, const double* __restrict__ cons,
                                                 const double* __restrict__ diagK, const double* __restrict__ Ktot,
                                                 const int* __restrict__ RU, TO* __restrict__ Pout,
                                                 TO* __restrict__ Psiout, double* __restrict__ Dout,
                                                 double* __restrict__ ScOut, int* __restrict__ flags) {
  constexpr int NU = 8 * P, NE = NU - 8, NCC = 4 * NCE, NC = 8 + NCC;
  constexpr int NSP = NU * (NU + 1) / 2;
  static_assert(NU <= 64, "one row per lane");
  const int cell = blockIdx.x, tid = threadIdx.x;
  // The first-stage arrays are dead once Psi is formed; S Psi takes the space
  // of A.  X, That and Chat are dead once P is formed, before Psi is written,
  // so the coarse basis takes theirs (the LDS of a workgroup then allows three
  // per CU in FP64 instead of two).
  struct Early {
    T X[NE][NCC + 1];    // Shat^-1 Chat^T
    T Tm[NCC][NCC + 1];  // That, then That^-1
    T Ch[NCC][NE];
  };
  struct Stage1 {
    T A[NE][NE + 1];     // Shat, then Shat^-1, then P
    T W2[NE][NCC + 1];   // X That^-1
    T Cc[NCC][8];
    T Scol[NE][8];
    union {
      Early e;
      double Ps[NU][NC + 1];  // coarse basis (unscaled)
    } tail;
  };
  union Work {
    Stage1 s;
    double SPs[NU][NC + 1];  // S Psi
  };
  static_assert(sizeof(double[NU][NC + 1]) <= sizeof(T[NE][NE + 1]) + sizeof(T[NE][NCC + 1]) +
                    sizeof(T[NCC][8]) + sizeof(T[NE][8]),
                "S Psi stays clear of the coarse basis it is formed from");
  __shared__ Work wk;
  __shared__ double Dv[NU];
  auto& Ps = wk.s.tail.Ps;
  __shared__ int bad;
  // clamped corners [0, 4) and clamped edges [4, 8) of the cell: their slots
  // have no global skeleton dof (Dirichlet), so they carry no constraint
  __shared__ int clamp[8];
  auto& A = wk.s.A;
  auto& X = wk.s.tail.e.X;
  auto& W2 = wk.s.W2;
  auto& Ch = wk.s.tail.e.Ch;
  auto& Cc = wk.s.Cc;
  auto& Tm = wk.s.tail.e.Tm;
  auto& Scol = wk.s.Scol;
  const double* S = Sg + (size_t)cell * NSP;
  if (tid == 0) bad = 0;
  // every global load of the cell first, from clamped positions (values past
  // the ranges are not used): the edge block of the packed S, its corner
  // columns, the weights' diagonals, the constraint rows
  constexpr int NLA = (NE * NE + 255) / 256, NLS = (NE * 8 + 255) / 256;
  constexpr int NCV = 4 * NCE * (P + 1) * 2;
  static_assert(NU <= 256 && NCV <= 256, "one weight and one constraint value per thread");
  // the index map first: the weight's denominator is gathered through it
  const int gw = tid < NU ? RU[(size_t)cell * NU + tid] : -1;
  double va[NLA], vs[NLS];
#pragma unroll
  for (int m = 0; m < NLA; ++m) {
    const int idx = tid + 256 * m < NE * NE ? tid + 256 * m : 0;
    const int I = 8 + idx / NE, J = 8 + idx % NE;
    const int hi = I > J ? I : J, lo = I > J ? J : I;
    va[m] = S[hi * (hi + 1) / 2 + lo];
  }
#pragma unroll
  for (int m = 0; m < NLS; ++m) {
    const int idx = tid + 256 * m < NE * 8 ? tid + 256 * m : 0;
    const int I = 8 + idx / 8;
    vs[m] = S[I * (I + 1) / 2 + idx % 8];
  }
  const double dk = diagK[(size_t)cell * NU + (tid < NU ? tid : 0)];
  const double* cc = cons + (size_t)cell * 4 * NCE * (P + 1) * 2;
  const double cv = cc[tid < NCV ? tid : 0];
  const double kt = Ktot[gw >= 0 ? gw : 0];
#pragma unroll
  for (int m = 0; m < NLA; ++m) {
    const int idx = tid + 256 * m;
    if (idx < NE * NE) A[idx / NE][idx % NE] = (T)va[m];
  }
#pragma unroll
  for (int m = 0; m < NLS; ++m) {
    const int idx = tid + 256 * m;
    if (idx < NE * 8) Scol[idx / 8][idx % 8] = (T)vs[m];
  }
  if (tid < NU) Dv[tid] = gw >= 0 ? dk / kt : 0.0;
  if (tid < 8 && (tid & 1) == 0) clamp[tid >> 1] = gw < 0;                  // corner node tid/2, x slot
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (tid == 2 * (4 + e * (P - 1))) clamp[4 + e] = gw < 0;                   // first interior node of edge e
  // constraint rows: Chat (edge dofs) and the corner columns
  for (int idx = tid; idx < NCC * NE; idx += 256) Ch[idx / NE][idx % NE] = (T)0;
  for (int idx = tid; idx < NCC * 8; idx += 256) Cc[idx / 8][idx % 8] = (T)0;
  __syncthreads();
  for (int idx = tid; idx < NCV; idx += 256) {
    const int comp = idx & 1, n = (idx >> 1) % (P + 1), et = (idx >> 1) / (P + 1);
    const int e = et / NCE;
    if (clamp[4 + e]) continue;  // a clamped edge carries no constraints
    const T v = (T)cv;
    if (n == 0 || n == P) {
      int corner = (e == 0) ? (n == 0 ? 0 : 2) : (e == 1) ? (n == 0 ? 1 : 3) : (e == 2) ? (n == 0 ? 0 : 1) : (n == 0 ? 2 : 3);
      if (clamp[corner]) continue;
      Cc[et][2 * corner + comp] = v;
    } else {
      Ch[et][2 * (e * (P - 1) + n - 1) + comp] = v;
    }
  }
  __syncthreads();
  // Shat^-1 in place
  gj_inverse_wave<T, NE + 1, NE>(&A[0][0], &bad);
  // X = Shat^-1 Chat^T
  mfma_mm<T, NE, NCC, NE>([&](int i, int k) { return A[i][k]; }, [&](int k, int a) { return Ch[a][k]; },
                          [&](int i, int a, T v) { X[i][a] = v; });
  __syncthreads();
  // That = Chat X; the rows of clamped edges carry no constraint and get a unit diagonal
  mfma_mm<T, NCC, NCC, NE>([&](int a, int i) { return Ch[a][i]; }, [&](int i, int b) { return X[i][b]; },
                           [&](int a, int b, T v) { Tm[a][b] = (a == b && clamp[4 + a / NCE]) ? (T)1 : v; });
  __syncthreads();
  gj_inverse_wave<T, NCC + 1, NCC>(&Tm[0][0], &bad);
  // W2 = X That^-1
  mfma_mm<T, NE, NCC, NCC>([&](int i, int b) { return X[i][b]; }, [&](int b, int a) { return Tm[b][a]; },
                           [&](int i, int a, T v) { W2[i][a] = v; });
  __syncthreads();
  // P = Shat^-1 - W2 X^T in place (each tile of A is read and written by one wave)
  mfma_mm<T, NE, NE, NCC>([&](int i, int a) { return W2[i][a]; }, [&](int a, int j) { return X[j][a]; },
                          [&](int i, int j, T v) { A[i][j] -= v; });
  __syncthreads();
  // store D_E P D_E packed lower
  TO* Pc = Pout + (size_t)cell * (NE * (NE + 1) / 2);
  for (int i = tid >> 6; i < NE; i += 4)
    for (int j = tid & 63; j <= i; j += 64)
      Pc[i * (i + 1) / 2 + j] = (TO)(Dv[8 + i] * (double)A[i][j] * Dv[8 + j]);
  // coarse basis Psi [NU][NC]: corner rows are the identity (masked for
  // clamped corners); edge rows: edge constraint columns W2, corner columns
  // -P S[E, c] - W2 C[:, c] (one product of depth NE + NCC)
  for (int idx = tid; idx < NU * NC; idx += 256) {
    const int i = idx / NC, j = idx % NC;
    const bool cmask = j < 8 && clamp[j >> 1];
    if (i < 8) {
      Ps[i][j] = (i == j && !cmask) ? 1.0 : 0.0;
    } else if (j >= 8) {
      const bool emask = clamp[4 + (j - 8) / NCE];
      Ps[i][j] = emask ? 0.0 : (double)W2[i - 8][j - 8];
    }
  }
  mfma_mm<T, NE, 8, NE + NCC>([&](int i, int k) { return k < NE ? A[i][k] : W2[i][k - NE]; },
                              [&](int k, int j) { return k < NE ? Scol[k][j] : Cc[k - NE][j]; },
                              [&](int i, int j, T v) {
                                const bool cmask = clamp[j >> 1];
                                Ps[8 + i][j] = cmask ? 0.0 : -(double)v;
                              });
  __syncthreads();
  // stored column by column, [NC][NU]: the PCG kernels read entry i of every
  // column in lane i
  TO* Pso = Psiout + (size_t)cell * NU * NC;
  for (int idx = tid; idx < NU * NC; idx += 256) {
    const int j = idx / NU, i = idx % NU;
    Pso[idx] = (TO)(Dv[i] * Ps[i][j]);
  }
  for (int j = tid; j < NU; j += 256) Dout[(size_t)cell * NU + j] = Dv[j];
  // S Psi in FP64 (S packed lower, read through the cache), then Psi^T S Psi;
  // S Psi overwrites the first-stage arrays (all reads of them ended at the
  // barrier above)
  mfma_mm<double, NU, NC, NU>(
      [&](int i, int k) {
        const int hi = i > k ? i : k, lo = i > k ? k : i;
        return S[hi * (hi + 1) / 2 + lo];
      },
      [&](int k, int j) { return Ps[k][j]; }, [&](int i, int j, double v) { wk.SPs[i][j] = v; });
  __syncthreads();
  double* Sc = ScOut + (size_t)cell * (NC * (NC + 1) / 2);
  mfma_mm<double, NC, NC, NU>([&](int a, int k) { return Ps[k][a]; }, [&](int k, int b) { return wk.SPs[k][b]; },
                              [&](int a, int b, double v) {
                                if (b <= a) Sc[a * (a + 1) / 2 + b] = v;
                              });
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

template <typename T, typename TO>
static hipError_t precond_T(Ctx* c) {
  dim3 grid(c->ncell), block(256);
  TO* Pout = (TO*)c->d_P;
  TO* Psi = (TO*)c->d_Psi;
#define PC_CASE(pp, ncv)                                                                                          \
  if (c->p == pp && c->nce == ncv) {                                                                             \
    hipLaunchKernelGGL((k_precond<T, TO, pp, ncv>), grid, block, 0, c->stream, c->d_S, c->d_cons, c->d_diagK,     \
                       c->d_Ktot, c->d_RU, Pout, Psi, c->d_D, c->d_ScLoc, c->d_flags);                    \
    return hipGetLastError();                                                                                    \
  }
  PC_CASE(2, 2) PC_CASE(2, 3) PC_CASE(3, 2) PC_CASE(3, 3) PC_CASE(4, 2) PC_CASE(4, 3) PC_CASE(5, 2) PC_CASE(5, 3)
  PC_CASE(6, 2) PC_CASE(6, 3) PC_CASE(7, 2) PC_CASE(7, 3) PC_CASE(8, 2) PC_CASE(8, 3)
#undef PC_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_precond(Ctx* c, bool fp32) {
  return fp32 ? precond_T<double, float>(c) : precond_T<double, double>(c);
}

}  // namespace lbddc
