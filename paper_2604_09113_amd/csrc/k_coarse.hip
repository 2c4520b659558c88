// Coarse problem S_C g = z (A8; the global coarse correction of Alg. 1).
//
// S_C = sum_i R_C^T (Psi^T S Psi) R_C is assembled deterministically (every
// entry the sum of its contributions in increasing cell order) straight into
// the frontal matrices of a nested-dissection tree of the cell grid (built on
// the host).  The exact FP64 factorization is multifrontal block LDL^T:
// bottom-up over the tree levels, each front F = [[F_ss, F_sb], [F_bs, F_bb]]
// (own dofs s, boundary dofs b) receives its children's update matrices
// (extend-add) and is swept by Gauss-Jordan over its own block, which leaves
//   [[F_ss^-1, M^T], [-M, U]],  M = F_bs F_ss^-1,  U = F_bb - M F_sb
// in place (F_ss is SPD, so no pivoting).  U goes to the parent.  A solve is a
// forward sweep up the tree, up = w_b - M b_eff (w_b: the children's
// contributions to the boundary dofs), and a backward sweep down the tree,
// g_s = F_ss^-1 b_eff - M^T g_b: one batched matrix-vector kernel per level
// and direction.
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

// extend-add of the update matrix of child slot `slot` of every node of a level
__global__ __launch_bounds__(256) void k_extend_add(const NDNodeH* __restrict__ nodes, const int* __restrict__ lvl,
                                                    const int* __restrict__ cmap, double* __restrict__ F, int slot) {
  const NDNodeH d = nodes[lvl[blockIdx.x]];
  const int ch = d.child[slot];
  if (ch < 0) return;
  const NDNodeH c = nodes[ch];
  const int nfc = c.ns + c.nb, nf = d.ns + d.nb;
  const int* map = cmap + d.cmap_off[slot];
  const double* U = F + c.foff;
  double* P = F + d.foff;
  for (long long idx = threadIdx.x; idx < (long long)c.nb * c.nb; idx += 256) {
    const int i = (int)(idx / c.nb), j = (int)(idx % c.nb);
    P[(long long)map[i] * nf + map[j]] += U[(long long)(c.ns + i) * nfc + c.ns + j];
  }
}

// Partial Gauss-Jordan sweep over the ns own dofs of small fronts: one
// workgroup per front, front in global memory, the pivot row and column staged
// in LDS each step (all updates read the pre-step values).
__global__ __launch_bounds__(256) void k_pgj_small(const NDNodeH* __restrict__ nodes, const int* __restrict__ lvl,
                                                   double* __restrict__ F, int* __restrict__ flags) {
  extern __shared__ double sh[];
  const NDNodeH d = nodes[lvl[blockIdx.x]];
  const int nf = d.ns + d.nb;
  double* A = F + d.foff;
  double* rowl = sh;
  double* coll = sh + nf;
  bool bad = false;
  for (int l = 0; l < d.ns; ++l) {
    for (int j = threadIdx.x; j < nf; j += 256) {
      rowl[j] = A[(long long)l * nf + j];
      coll[j] = A[(long long)j * nf + l];
    }
    __syncthreads();
    double piv = rowl[l];
    if (!(piv > 0.0)) { bad = true; piv = 1.0; }
    const double pinv = 1.0 / piv;
    for (long long idx = threadIdx.x; idx < (long long)nf * nf; idx += 256) {
      const int i = (int)(idx / nf), j = (int)(idx % nf);
      double v;
      if (i == l && j == l) v = pinv;
      else if (i == l) v = rowl[j] * pinv;
      else if (j == l) v = -coll[i] * pinv;
      else v = A[idx] - coll[i] * rowl[j] * pinv;
      A[idx] = v;
    }
    __syncthreads();
  }
  if (bad) atomicOr(flags, 32);
}

// ---- blocked Gauss-Jordan sweep over pivot rows [0, ns) of one large front ----
constexpr int GJB = 64;

// invert the kn x kn diagonal block at (k0, k0) into P [GJB][GJB] (identity padded)
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
      for (int a = 0; a < 4; ++a)
        if (a == la) {
#pragma unroll
          for (int bb = 0; bb < 4; ++bb) rowb[buf][tc + 16 * bb] = B[a][bb];
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

// R[l][j] = sum_q P[l][q] A[k0 + q][j] for every column j, and Cp[i][l] = A[i][k0 + l]
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
  for (int idx = t; idx < GJB * GJB; idx += 256) {
    int i = j0 + idx / GJB, l = idx % GJB;
    if (i < m && l < kn) Cp[(size_t)i * GJB + l] = A[(size_t)i * m + k0 + l];
  }
}

// element (i, j): pivot row and column -> P; pivot row -> R; pivot column ->
// -Cp P; otherwise A -= Cp R.  Tiles are 64 x 64; pivot rows are [k0, k0 + kn).
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, int m, int k0, int kn,
                                                   const double* __restrict__ P, const double* __restrict__ R,
                                                   const double* __restrict__ Cp) {
  __shared__ double Cs[GJB][GJB + 1];
  __shared__ double Rs[GJB][GJB + 1];
  const int t = threadIdx.x, i0 = blockIdx.y * GJB, j0 = blockIdx.x * GJB;
  for (int idx = t; idx < GJB * GJB; idx += 256) {
    int a = idx / GJB, b = idx % GJB;
    int i = i0 + a, j = j0 + b;
    Cs[a][b] = (i < m && b < kn) ? Cp[(size_t)i * GJB + b] : 0.0;
    Rs[a][b] = (a < kn && j < m) ? R[(size_t)a * m + j] : 0.0;
  }
  __syncthreads();
  const int tr = t >> 4, tc = t & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int li = tr + 16 * a, lj = tc + 16 * b, i = i0 + li, j = j0 + lj;
      if (i >= m || j >= m) continue;
      const bool ip = i >= k0 && i < k0 + kn, jp = j >= k0 && j < k0 + kn;
      if (ip && jp) {
        A[(size_t)i * m + j] = P[(i - k0) * GJB + (j - k0)];
      } else if (ip) {
        A[(size_t)i * m + j] = Rs[i - k0][lj];
      } else if (jp) {
        double s = 0.0;
        for (int q = 0; q < kn; ++q) s += Cs[li][q] * P[q * GJB + (j - k0)];
        A[(size_t)i * m + j] = -s;
      } else {
        double s = 0.0;
        for (int q = 0; q < kn; ++q) s += Cs[li][q] * Rs[q][lj];
        A[(size_t)i * m + j] -= s;
      }
    }
}

static hipError_t gj_partial(Ctx* c, double* A, int m, int npiv) {
  const int nblk = (m + GJB - 1) / GJB;
  for (int k0 = 0; k0 < npiv; k0 += GJB) {
    const int kn = std::min(GJB, npiv - k0);
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, c->stream, A, m, k0, kn, c->d_gjP, c->d_flags);
    hipLaunchKernelGGL(k_gj_panel, dim3(nblk), dim3(256), 0, c->stream, A, m, k0, kn, c->d_gjP, c->d_gjR, c->d_gjC);
    hipLaunchKernelGGL(k_gj_update, dim3(nblk, nblk), dim3(256), 0, c->stream, A, m, k0, kn, c->d_gjP, c->d_gjR,
                       c->d_gjC);
  }
  return hipGetLastError();
}

hipError_t launch_coarse_assemble(Ctx* c) {
  const CoarseLayout& co = c->co;
  hipLaunchKernelGGL(k_fill, dim3(2048), dim3(256), 0, c->stream, c->d_coarse, co.nd_front_total, 0.0);
  int nent = (int)co.dest.size();
  hipLaunchKernelGGL(k_coarse_entries, dim3((nent + 255) / 256), dim3(256), 0, c->stream, c->d_ScLoc, c->d_cstart,
                     c->d_contrib, c->d_dest, c->d_coarse, nent);
  return hipGetLastError();
}

hipError_t launch_coarse_factor(Ctx* c) {
  const CoarseLayout& co = c->co;
  for (int l = (int)co.nd_levels.size() - 1; l >= 0; --l) {
    const int n0 = co.lvl_off[l], nn = co.lvl_off[l + 1] - n0;
    const int* lvl = c->d_lvl_nodes + n0;
    for (int s = 0; s < 2; ++s)
      hipLaunchKernelGGL(k_extend_add, dim3(nn), dim3(256), 0, c->stream, c->d_nd_nodes, lvl, c->d_nd_cmap,
                         c->d_coarse, s);
    int nfmax = 0;
    for (int n : co.nd_levels[l]) nfmax = std::max(nfmax, co.nd_nodes[n].ns + co.nd_nodes[n].nb);
    if (nn >= 32) {
      hipLaunchKernelGGL(k_pgj_small, dim3(nn), dim3(256), 2 * nfmax * sizeof(double), c->stream, c->d_nd_nodes,
                         lvl, c->d_coarse, c->d_flags);
    } else {
      for (int n : co.nd_levels[l]) {
        const NDNodeH& d = co.nd_nodes[n];
        hipError_t e = gj_partial(c, c->d_coarse + d.foff, d.ns + d.nb, d.ns);
        if (e != hipSuccess) return e;
      }
    }
  }
  return hipGetLastError();
}

// forward sweep of one level: item = (node, first boundary row)
__global__ __launch_bounds__(256) void k_nd_fwd(const NDNodeH* __restrict__ nodes, const int* __restrict__ items,
                                                const int* __restrict__ own, const int* __restrict__ cmap,
                                                const double* __restrict__ F, const double* __restrict__ b,
                                                double* __restrict__ up, double* __restrict__ beff) {
  extern __shared__ double sh[];
  const int nid = items[2 * blockIdx.x], r0 = items[2 * blockIdx.x + 1];
  const NDNodeH d = nodes[nid];
  const int nf = d.ns + d.nb;
  double* w = sh;        // [nf] children's contributions
  double* be = sh + nf;  // [ns]
  for (int i = threadIdx.x; i < nf; i += 256) w[i] = 0.0;
  __syncthreads();
  for (int s = 0; s < 2; ++s) {
    const int ch = d.child[s];
    if (ch >= 0) {
      const NDNodeH c = nodes[ch];
      const int* map = cmap + d.cmap_off[s];
      for (int i = threadIdx.x; i < c.nb; i += 256) w[map[i]] += up[c.up_off + i];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < d.ns; i += 256) {
    const double v = b[own[d.own_off + i]] + w[i];
    be[i] = v;
    if (r0 == 0) beff[d.beff_off + i] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, r = r0 + (threadIdx.x >> 6);
  if (r >= d.nb) return;
  const double* row = F + d.foff + (long long)(d.ns + r) * nf;  // -M
  double s = 0.0;
  for (int k = lane; k < d.ns; k += 64) s += row[k] * be[k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) up[d.up_off + r] = w[d.ns + r] + s;
}

// backward sweep of one level: item = (node, first own row); g_s = [F_ss^-1 | M^T] [b_eff; -g_b]
__global__ __launch_bounds__(256) void k_nd_bwd(const NDNodeH* __restrict__ nodes, const int* __restrict__ items,
                                                const int* __restrict__ own, const int* __restrict__ bnd,
                                                const double* __restrict__ F, const double* __restrict__ beff,
                                                double* __restrict__ x) {
  extern __shared__ double sh[];
  const int nid = items[2 * blockIdx.x], r0 = items[2 * blockIdx.x + 1];
  const NDNodeH d = nodes[nid];
  const int nf = d.ns + d.nb;
  for (int i = threadIdx.x; i < nf; i += 256)
    sh[i] = i < d.ns ? beff[d.beff_off + i] : -x[bnd[d.bnd_off + i - d.ns]];
  __syncthreads();
  const int lane = threadIdx.x & 63, r = r0 + (threadIdx.x >> 6);
  if (r >= d.ns) return;
  const double* row = F + d.foff + (long long)r * nf;
  double s = 0.0;
  for (int k = lane; k < nf; k += 64) s += row[k] * sh[k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) x[own[d.own_off + r]] = s;
}

hipError_t launch_coarse_solve(Ctx* c, const double* rhs, double* x) {
  const CoarseLayout& co = c->co;
  const size_t lds_f = (size_t)(co.nd_nfmax + co.nd_nsmax) * sizeof(double);
  const size_t lds_b = (size_t)co.nd_nfmax * sizeof(double);
  const int L = (int)co.nd_levels.size();
  for (int l = L - 1; l >= 0; --l) {
    const int i0 = co.fw_off[l], ni = co.fw_off[l + 1] - i0;
    if (ni > 0)
      hipLaunchKernelGGL(k_nd_fwd, dim3(ni), dim3(256), lds_f, c->stream, c->d_nd_nodes, c->d_fw_items + 2 * i0,
                         c->d_nd_own, c->d_nd_cmap, c->d_coarse, rhs, c->d_up, c->d_beff);
  }
  for (int l = 0; l < L; ++l) {
    const int i0 = co.bw_off[l], ni = co.bw_off[l + 1] - i0;
    if (ni > 0)
      hipLaunchKernelGGL(k_nd_bwd, dim3(ni), dim3(256), lds_b, c->stream, c->d_nd_nodes, c->d_bw_items + 2 * i0,
                         c->d_nd_own, c->d_nd_bnd, c->d_coarse, c->d_beff, x);
  }
  return hipGetLastError();
}

}  // namespace lbddc
