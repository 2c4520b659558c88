// Coarse problem S_C g = z (A8; Sec. 3.3.4, the global coarse correction).
//
// S_C = sum_i R_C^T (Psi^T S Psi) R_C is assembled deterministically: every
// nonzero of S_C is the sum of its contributions in increasing cell order.  In
// the grid-line ordering of the coarse dofs S_C is block tridiagonal with
// diagonal blocks A_j (dense) and sparse couplings B_j = A[j+1, j].  The exact
// FP64 factorization is the block Thomas recursion
//   D_0 = A_0,  D_j = A_j - B_{j-1} D_{j-1}^-1 B_{j-1}^T,
// keeping D_j^-1 explicitly (in-place blocked Gauss-Jordan; the D_j are SPD,
// so no pivoting is needed), and each coarse solve is two sweeps of dense
// matrix-vector products with D_j^-1 and sparse products with B_j:
//   forward  t_j = D_j^-1 (z_j - B_{j-1} t_{j-1})
//   backward g_j = t_j - D_j^-1 B_j^T g_{j+1}.
#include "internal.h"

namespace lbddc {

__global__ void k_fill(double* __restrict__ x, long long n, double v) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) x[i] = v;
}

__global__ void k_coarse_entries(const double* __restrict__ sc, const int* __restrict__ cstart,
                                 const int* __restrict__ contrib, const long long* __restrict__ dest,
                                 double* __restrict__ vals, int nent) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  double s = 0.0;
  for (int i = cstart[e]; i < cstart[e + 1]; ++i) s += sc[contrib[i]];
  vals[dest[e]] = s;
}

// W[a][c] = sum_{(k,v) in row c of B} Dinv[a][k] v      (W = Dinv B^T, m0 x m1)
__global__ void k_coarse_W(const double* __restrict__ Dinv, int m0, const int* __restrict__ rp,
                           const int* __restrict__ col, const double* __restrict__ val, int m1,
                           double* __restrict__ W) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)m0 * m1) return;
  int a = (int)(id / m1), c = (int)(id % m1);
  double s = 0.0;
  for (int o = rp[c]; o < rp[c + 1]; ++o) s += Dinv[(size_t)a * m0 + col[o]] * val[o];
  W[id] = s;
}

// D[r][c] -= sum_{(k,v) in row r of B} v W[k][c]
__global__ void k_coarse_update(double* __restrict__ D, int m1, const int* __restrict__ rp,
                                const int* __restrict__ col, const double* __restrict__ val,
                                const double* __restrict__ W) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)m1 * m1) return;
  int r = (int)(id / m1), c = (int)(id % m1);
  double s = 0.0;
  for (int o = rp[r]; o < rp[r + 1]; ++o) s += val[o] * W[(size_t)col[o] * m1 + c];
  D[id] -= s;
}

// ---- in-place blocked Gauss-Jordan inversion of an SPD matrix (row-major) ----
constexpr int GJB = 64;

// Invert the kn x kn diagonal block at (k0, k0) in registers + LDS broadcast;
// write the inverse to P [GJB][GJB].
__global__ __launch_bounds__(256) void k_gj_diag(const double* __restrict__ A, int m, int k0, int kn,
                                                 double* __restrict__ P, int* __restrict__ flags) {
  __shared__ double rowb[2][GJB], colb[2][GJB];
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  double B[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int i = tr + 16 * a, j = tc + 16 * b;
      B[a][b] = (i < kn && j < kn) ? A[(size_t)(k0 + i) * m + k0 + j] : (i == j ? 1.0 : 0.0);
    }
  int buf = 0;
  bool bad = false;
  for (int l = 0; l < GJB; ++l) {
    const int la = l >> 4, lb = l & 15;
    if (tr == lb) {
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b == la) {
#pragma unroll
          for (int bb = 0; bb < 4; ++bb) rowb[buf][tc + 16 * bb] = B[b][bb];
        }
    }
    if (tc == lb) {
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b == la) {
#pragma unroll
          for (int a = 0; a < 4; ++a) colb[buf][tr + 16 * a] = B[a][b];
        }
    }
    __syncthreads();
    double piv = rowb[buf][l];
    if (!(piv > 0.0)) { bad = true; piv = 1.0; }
    const double pinv = 1.0 / piv;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        int i = tr + 16 * a, j = tc + 16 * b;
        double v = B[a][b];
        if (i == l && j == l) v = pinv;
        else if (i == l) v = v * pinv;
        else if (j == l) v = -v * pinv;
        else v = v - colb[buf][i] * rowb[buf][j] * pinv;
        B[a][b] = v;
      }
    buf ^= 1;
  }
  if (bad) atomicOr(flags, 32);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) P[(tr + 16 * a) * GJB + tc + 16 * b] = B[a][b];
}

// R[l][j] = sum_l' P[l][l'] A[k0 + l'][j] for every column j (block columns
// included; the update kernel ignores them), and Cp[i][l] = A[i][k0 + l].
__global__ __launch_bounds__(256) void k_gj_panel(const double* __restrict__ A, int m, int k0, int kn,
                                                  const double* __restrict__ P, double* __restrict__ R,
                                                  double* __restrict__ Cp) {
  __shared__ double Ps[GJB][GJB + 1];
  __shared__ double As[GJB][GJB + 1];
  const int t = threadIdx.x, j0 = blockIdx.x * GJB;
  for (int idx = t; idx < GJB * GJB; idx += 256) {
    int a = idx / GJB, b = idx % GJB;
    Ps[a][b] = P[idx];
    int j = j0 + b;
    As[a][b] = (a < kn && j < m) ? A[(size_t)(k0 + a) * m + j] : 0.0;
  }
  __syncthreads();
  for (int idx = t; idx < GJB * GJB; idx += 256) {
    int l = idx / GJB, b = idx % GJB, j = j0 + b;
    if (l >= kn || j >= m) continue;
    double s = 0.0;
    for (int q = 0; q < kn; ++q) s += Ps[l][q] * As[q][b];
    R[(size_t)l * m + j] = s;
  }
  // column panel copy of rows [j0, j0 + 64)
  for (int idx = t; idx < GJB * GJB; idx += 256) {
    int i = j0 + idx / GJB, l = idx % GJB;
    if (i < m && l < kn) Cp[(size_t)i * GJB + l] = A[(size_t)i * m + k0 + l];
  }
}

__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, int m, int k0, int kn,
                                                   const double* __restrict__ P, const double* __restrict__ R,
                                                   const double* __restrict__ Cp) {
  __shared__ double Cs[GJB][GJB + 1];
  __shared__ double Rs[GJB][GJB + 1];
  const int t = threadIdx.x, i0 = blockIdx.y * GJB, j0 = blockIdx.x * GJB;
  const bool rowk = (i0 == k0), colk = (j0 == k0);
  for (int idx = t; idx < GJB * GJB; idx += 256) {
    int a = idx / GJB, b = idx % GJB;
    int i = i0 + a, j = j0 + b;
    Cs[a][b] = (i < m && b < kn) ? Cp[(size_t)i * GJB + b] : 0.0;
    if (colk) Rs[a][b] = P[a * GJB + b];  // right factor of -Cp P
    else Rs[a][b] = (a < kn && j < m) ? R[(size_t)a * m + j] : 0.0;
  }
  __syncthreads();
  const int tr = t >> 4, tc = t & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int li = tr + 16 * a, lj = tc + 16 * b, i = i0 + li, j = j0 + lj;
      if (i >= m || j >= m) continue;
      if (rowk && colk) {
        if (li < kn && lj < kn) A[(size_t)i * m + j] = P[li * GJB + lj];
      } else if (rowk) {
        if (li < kn) A[(size_t)i * m + j] = R[(size_t)li * m + j];
      } else if (colk) {
        if (lj < kn) {
          double s = 0.0;
          for (int q = 0; q < kn; ++q) s += Cs[li][q] * Rs[q][lj];
          A[(size_t)i * m + j] = -s;
        }
      } else {
        double s = 0.0;
        for (int q = 0; q < kn; ++q) s += Cs[li][q] * Rs[q][lj];
        A[(size_t)i * m + j] -= s;
      }
    }
}

static hipError_t gj_invert(Ctx* c, double* A, int m) {
  const int nblk = (m + GJB - 1) / GJB;
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * GJB, kn = std::min(GJB, m - k0);
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, c->stream, A, m, k0, kn, c->d_gjP, c->d_flags);
    hipLaunchKernelGGL(k_gj_panel, dim3(nblk), dim3(256), 0, c->stream, A, m, k0, kn, c->d_gjP, c->d_gjR, c->d_gjC);
    hipLaunchKernelGGL(k_gj_update, dim3(nblk, nblk), dim3(256), 0, c->stream, A, m, k0, kn, c->d_gjP, c->d_gjR,
                       c->d_gjC);
  }
  return hipGetLastError();
}

hipError_t launch_coarse_assemble(Ctx* c) {
  const CoarseLayout& co = c->co;
  long long ntot = co.dense_total + co.nnzB + co.nnzBT;
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, c->stream, c->d_coarse, ntot, 0.0);
  int nent = (int)co.dest.size();
  hipLaunchKernelGGL(k_coarse_entries, dim3((nent + 255) / 256), dim3(256), 0, c->stream, c->d_ScLoc, c->d_cstart,
                     c->d_contrib, c->d_dest, c->d_coarse, nent);
  return hipGetLastError();
}

hipError_t launch_coarse_factor(Ctx* c) {
  const CoarseLayout& co = c->co;
  double* dense = c->d_coarse;
  const double* bval = c->d_coarse + co.dense_total;
  for (int j = 0; j < co.nsb; ++j) {
    const int m1 = co.sb_size[j];
    double* Dj = dense + co.dense_off[j];
    if (j > 0) {
      const int m0 = co.sb_size[j - 1];
      const double* Dprev = dense + co.dense_off[j - 1];
      const int* rp = c->d_b_rowptr + co.b_rowptr_off[j - 1];
      const int* cl = c->d_b_col + co.b_val_off[j - 1];
      const double* vv = bval + co.b_val_off[j - 1];
      long long nW = (long long)m0 * m1;
      hipLaunchKernelGGL(k_coarse_W, dim3((unsigned)((nW + 255) / 256)), dim3(256), 0, c->stream, Dprev, m0, rp, cl,
                         vv, m1, c->d_gjW);
      long long nD = (long long)m1 * m1;
      hipLaunchKernelGGL(k_coarse_update, dim3((unsigned)((nD + 255) / 256)), dim3(256), 0, c->stream, Dj, m1, rp,
                         cl, vv, c->d_gjW);
    }
    hipError_t e = gj_invert(c, Dj, m1);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// forward step j: y = z_j - B_{j-1} t_{j-1} (redundant per workgroup), t_j = Dinv_j y
__global__ __launch_bounds__(256) void k_cs_fwd(const double* __restrict__ Dinv, int m, const double* __restrict__ z,
                                                double* __restrict__ t, int off, int offp,
                                                const int* __restrict__ rp, const int* __restrict__ col,
                                                const double* __restrict__ val, int has_prev,
                                                double* __restrict__ xlast) {
  extern __shared__ double y[];
  for (int a = threadIdx.x; a < m; a += 256) {
    double s = z[off + a];
    if (has_prev)
      for (int o = rp[a]; o < rp[a + 1]; ++o) s -= val[o] * t[offp + col[o]];
    y[a] = s;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = blockIdx.x * 4 + wave;
  if (r >= m) return;
  const double* row = Dinv + (size_t)r * m;
  double s = 0.0;
  for (int a = lane; a < m; a += 64) s += row[a] * y[a];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) {
    t[off + r] = s;
    if (xlast) xlast[off + r] = s;
  }
}

// backward step j: v = B_j^T g_{j+1}, g_j = t_j - Dinv_j v
__global__ __launch_bounds__(256) void k_cs_bwd(const double* __restrict__ Dinv, int m, const double* __restrict__ t,
                                                double* __restrict__ g, int off, int offn,
                                                const int* __restrict__ rp, const int* __restrict__ col,
                                                const double* __restrict__ val) {
  extern __shared__ double v[];
  for (int a = threadIdx.x; a < m; a += 256) {
    double s = 0.0;
    for (int o = rp[a]; o < rp[a + 1]; ++o) s += val[o] * g[offn + col[o]];
    v[a] = s;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = blockIdx.x * 4 + wave;
  if (r >= m) return;
  const double* row = Dinv + (size_t)r * m;
  double s = 0.0;
  for (int a = lane; a < m; a += 64) s += row[a] * v[a];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) g[off + r] = t[off + r] - s;
}

hipError_t launch_coarse_solve(Ctx* c, const double* rhs, double* x) {
  const CoarseLayout& co = c->co;
  const double* dense = c->d_coarse;
  const double* bval = c->d_coarse + co.dense_total;
  const double* btval = c->d_coarse + co.dense_total + co.nnzB;
  for (int j = 0; j < co.nsb; ++j) {
    const int m = co.sb_size[j];
    const int hp = j > 0;
    const int* rp = hp ? c->d_b_rowptr + co.b_rowptr_off[j - 1] : c->d_b_rowptr;
    const int* cl = hp ? c->d_b_col + co.b_val_off[j - 1] : c->d_b_col;
    const double* vv = hp ? bval + co.b_val_off[j - 1] : bval;
    hipLaunchKernelGGL(k_cs_fwd, dim3((m + 3) / 4), dim3(256), m * sizeof(double), c->stream,
                       dense + co.dense_off[j], m, rhs, c->d_tc, co.sb_off[j], hp ? co.sb_off[j - 1] : 0, rp, cl, vv,
                       hp, j == co.nsb - 1 ? x : (double*)nullptr);
  }
  for (int j = co.nsb - 2; j >= 0; --j) {
    const int m = co.sb_size[j];
    hipLaunchKernelGGL(k_cs_bwd, dim3((m + 3) / 4), dim3(256), m * sizeof(double), c->stream,
                       dense + co.dense_off[j], m, c->d_tc, x, co.sb_off[j], co.sb_off[j + 1],
                       c->d_bt_rowptr + co.bt_rowptr_off[j], c->d_bt_col + co.bt_val_off[j], btval + co.bt_val_off[j]);
  }
  return hipGetLastError();
}

}  // namespace lbddc
