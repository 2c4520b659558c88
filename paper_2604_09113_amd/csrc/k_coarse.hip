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
#include "wave_gj.h"

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

// extend-add of the update matrix of child slot `slot` of every node of a level;
// KC column chunks of 64 per lane cover the level's largest child boundary
// (KC = 0: boundaries past 1024 columns, a plain strided loop)
template <int KC>
__global__ __launch_bounds__(256) void k_extend_add(const NDNodeH* __restrict__ nodes, const int* __restrict__ lvl,
                                                    const int* __restrict__ cmap, double* __restrict__ F, int slot) {
  const NDNodeH d = nodes[lvl[blockIdx.x]];
  const int r0 = 16 * blockIdx.y;
  const int ch = d.child[slot];
  if (ch < 0) return;
  const NDNodeH c = nodes[ch];
  const int nfc = c.ns + c.nb, nf = d.ns + d.nb, nb = c.nb;
  const int* map = cmap + d.cmap_off[slot];
  const double* U = F + c.foff;
  double* P = F + d.foff;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rend = min(nb, r0 + 16);
  if constexpr (KC == 0) {
    for (int i = r0 + wave; i < rend; i += 4) {
      double* prow = P + (long long)map[i] * nf;
      const double* urow = U + (long long)(c.ns + i) * nfc + c.ns;
      for (int j = lane; j < nb; j += 64) prow[map[j]] += urow[j];
    }
    return;
  } else {
    // the map entries of the lane's columns and of the wave's rows first; then
    // every load of RB rows before any add (columns past nb and rows past the
    // block read the position of column or row 0 and are not stored)
    constexpr int RB = KC <= 4 ? 4 : 1;  // rows in flight together
    int mj[KC], mi[4];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int j = lane + 64 * k;
      mj[k] = map[j < nb ? j : 0];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = r0 + wave + 4 * q;
      mi[q] = map[i < rend ? i : 0];
    }
#pragma unroll
    for (int q0 = 0; q0 < 4; q0 += RB) {
      double u[RB][KC], pv[RB][KC];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int i = r0 + wave + 4 * (q0 + q), ic = i < rend ? i : r0;
        const double* prow = P + (long long)mi[q0 + q] * nf;
        const double* urow = U + (long long)(c.ns + ic) * nfc + c.ns;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
          const int j = lane + 64 * k;
          u[q][k] = urow[j < nb ? j : 0];
          pv[q][k] = prow[mj[k]];
        }
      }
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int i = r0 + wave + 4 * (q0 + q);
        if (i < rend) {
          double* prow = P + (long long)mi[q0 + q] * nf;
#pragma unroll
          for (int k = 0; k < KC; ++k)
            if (lane + 64 * k < nb) prow[mj[k]] = pv[q][k] + u[q][k];
        }
      }
    }
  }
}

// ---- Gauss-Jordan sweep of a front over its own dofs ----
//
// Small fronts (nf <= ND_LDS_NF, the lower tree levels) are swept one
// workgroup per front with the whole front resident in LDS: load, add the
// children's update matrices, eliminate the ns pivots one by one, store.
//
// Larger fronts (upper levels: few nodes, fronts of several hundred dofs) are
// swept in pivot blocks K = [k0, k0 + kn), kn <= 64, every front of the level
// in the same launch, three kernels per block:
//   diag   F[K][K] <- F[K][K]^-1                              (one WG per front)
//   panel  F[K][j] <- F[K][K]^-1 F[K][j] for j outside K,
//          Cp[i] <- F[i][K] for i outside K                    (column tiles)
//   update F[i][j] -= Cp[i] F[K][j], F[i][K] <- -Cp[i] F[K][K]  (64 x 64 tiles)
// which is the same elimination as the pivot-by-pivot sweep, regrouped.
constexpr int GJB = 64;

template <int NF, int NT>
__global__ __launch_bounds__(NT) void k_front_lds(const NDNodeH* __restrict__ nodes, const int* __restrict__ lvl,
                                                  const int* __restrict__ cmap, double* __restrict__ F,
                                                  int* __restrict__ flags) {
  constexpr int W = NT / 64;  // waves
  __shared__ double S[NF * (NF + 1)];
  __shared__ double rowl[NF], coll[NF];
  const NDNodeH d = nodes[lvl[blockIdx.x]];
  const int nf = d.ns + d.nb, ld = nf + 1;
  double* A = F + d.foff;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NR = (NF + W - 1) / W, NJ0 = (NF + 63) / 64;  // rows per wave, column chunks
  // the thread's entries of the front, every load in flight together: the
  // row address advances in a per-lane pointer (rows past nf re-read the last
  // row, columns past nf read column 0; neither is stored)
  {
    double v[NR][NJ0];
    const double* pr = A + (wave < nf ? (long long)wave * nf : 0);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
#pragma unroll
      for (int c = 0; c < NJ0; ++c) v[k][c] = pr[lane + 64 * c < nf ? lane + 64 * c : 0];
      pr += wave + W * (k + 1) < nf ? (long long)W * nf : 0;
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int i = wave + W * k;
      if (i >= nf) break;
#pragma unroll
      for (int c = 0; c < NJ0; ++c)
        if (lane + 64 * c < nf) S[i * ld + lane + 64 * c] = v[k][c];
    }
  }
  __syncthreads();
  for (int s = 0; s < 2; ++s) {
    const int ch = d.child[s];
    if (ch < 0) continue;
    const NDNodeH c = nodes[ch];
    const int nfc = c.ns + c.nb, nb = c.nb;
    const int* map = cmap + d.cmap_off[s];
    const double* U = F + c.foff + (long long)c.ns * nfc + c.ns;
    // the child's update rows are at most nf long: the map entries and the
    // values are all requested before the adds
    int mj[NJ0], mi[NR];
    double u[NR][NJ0];
#pragma unroll
    for (int cc = 0; cc < NJ0; ++cc) mj[cc] = map[lane + 64 * cc < nb ? lane + 64 * cc : 0];
    const double* ur = U + (wave < nb ? (long long)wave * nfc : 0);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int i = wave + W * k;
      mi[k] = map[i < nb ? i : 0];
#pragma unroll
      for (int cc = 0; cc < NJ0; ++cc) u[k][cc] = ur[lane + 64 * cc < nb ? lane + 64 * cc : 0];
      ur += i + W < nb ? (long long)W * nfc : 0;
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (wave + W * k >= nb) break;
      const int r = mi[k] * ld;
#pragma unroll
      for (int cc = 0; cc < NJ0; ++cc)
        if (lane + 64 * cc < nb) S[r + mj[cc]] += u[k][cc];
    }
    __syncthreads();
  }
  bool bad = false;
  constexpr int NJ = (NF + 63) / 64;  // row chunks of 64 columns
  for (int l = 0; l < d.ns; ++l) {
    for (int j = threadIdx.x; j < nf; j += NT) {
      rowl[j] = S[l * ld + j];
      coll[j] = S[j * ld + l];
    }
    __syncthreads();
    double piv = rowl[l];
    if (!(piv > 0.0)) { bad = true; piv = 1.0; }
    const double pinv = recip_refined(piv);
    // loads are unconditional (columns past nf read column 0 and are not
    // stored), so the loads of a row pair are all in flight before the updates
    double rv[NJ];  // this lane's columns of the pivot row
#pragma unroll
    for (int c = 0; c < NJ; ++c) rv[c] = rowl[lane + 64 * c < nf ? lane + 64 * c : 0];
    // rows i and i + W per iteration; the pivot row is scaled by 1/p (1/p on the
    // diagonal), the others become s - (c_i / p) r_j (-c_i / p in the pivot column)
    for (int i = wave; i < nf; i += 2 * W) {
      const int i2 = i + W;
      const bool has2 = i2 < nf;
      double* r1 = S + i * ld;
      double* r2 = S + (has2 ? i2 : i) * ld;
      double s1[NJ], s2[NJ];
#pragma unroll
      for (int c = 0; c < NJ; ++c) {
        const int j = lane + 64 * c < nf ? lane + 64 * c : 0;
        s1[c] = r1[j];
        s2[c] = r2[j];
      }
      const double c1 = coll[i] * pinv, c2 = coll[has2 ? i2 : i] * pinv;
#pragma unroll
      for (int c = 0; c < NJ; ++c) {
        const int j = lane + 64 * c;
        if (j < nf) {
          r1[j] = i == l ? (j == l ? pinv : rv[c] * pinv) : (j == l ? -c1 : s1[c] - c1 * rv[c]);
          if (has2) r2[j] = i2 == l ? (j == l ? pinv : rv[c] * pinv) : (j == l ? -c2 : s2[c] - c2 * rv[c]);
        }
      }
    }
    __syncthreads();
  }
  for (int i = wave; i < nf; i += W)
    for (int j = lane; j < nf; j += 64) A[(long long)i * nf + j] = S[i * ld + j];
  if (bad) atomicOr(flags, 32);
}

// Inversion of the kn x kn diagonal block at A (row stride nf), identity
// padded to 64 x 64, by a Gauss-Jordan sweep regrouped into four 16-pivot
// blocks.  The block is held in LDS.  For pivot block K (rows and columns
// [16 kb, 16 kb + 16)):
//   D <- D^-1                     (D = M[K][K]; one wave, in registers)
//   R  = D M[K][j]                (the new pivot rows, j outside K)
//   M[i][j] <- M[i][j] - M[i][K] R,  M[i][K] <- -M[i][K] D,  M[K][j] <- R
//                                 (i, j outside K)
// which is the same elimination as sixteen single-pivot steps.  The 16 x 16
// tile products run on FP64 MFMA, one tile per wave.  Pivot blocks that lie
// wholly in the padding are skipped (they would leave it unchanged).
constexpr int DLD = GJB + 1;  // LDS row stride of the block

// 16 x 16 tile product on MFMA 16x16x4 (FP64): lane l supplies a(m, k) and
// b(k, n) with m = n = l % 16, k = l / 16 + 4 s, and receives C[l / 16 + 4 v][l % 16]
// in value v of the result.
typedef double dbl4c __attribute__((ext_vector_type(4)));
template <typename FA, typename FB>
__device__ __forceinline__ dbl4c tile16(FA a, FB b) {
  const int lane = threadIdx.x & 63, mn = lane & 15, kk = lane >> 4;
  dbl4c acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a(mn, kk + 4 * s), b(kk + 4 * s, mn), acc, 0, 0, 0);
  return acc;
}

__global__ __launch_bounds__(256) void k_lv_diag(const NDNodeH* __restrict__ nodes, const int* __restrict__ lvl,
                                                 double* __restrict__ F, int k0, int* __restrict__ flags) {
  __shared__ double M[GJB * DLD];
  __shared__ double R[16 * DLD];
  __shared__ int bad;
  const NDNodeH d = nodes[lvl[blockIdx.x]];
  if (k0 >= d.ns) return;
  const int kn = min(GJB, d.ns - k0), nf = d.ns + d.nb;
  double* A = F + d.foff + (long long)k0 * nf + k0;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  // every load in flight before the identity padding is applied
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = (t >> 6) + 4 * q, j = t & 63;
    v[q] = A[(long long)(i < kn ? i : 0) * nf + (j < kn ? j : 0)];
  }
  if (t == 0) bad = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = (t >> 6) + 4 * q, j = t & 63;
    M[i * DLD + j] = (i < kn && j < kn) ? v[q] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int row = lane >> 4, col = lane & 15;  // result value u sits at (row + 4u, col)
  for (int kb = 0; 16 * kb < kn; ++kb) {
    const int K0 = 16 * kb;
    gj_inverse_wave<double, DLD, 16>(M + K0 * DLD + K0, &bad);  // ends with a barrier
    // R = D^-1 M[K][jb] for the three column blocks jb != kb (waves 0-2)
    if (wave < 3) {
      const int jb = wave + (wave >= kb);
      const dbl4c r = tile16([&](int m, int k) { return M[(K0 + m) * DLD + K0 + k]; },
                             [&](int k, int n) { return M[(K0 + k) * DLD + 16 * jb + n]; });
#pragma unroll
      for (int u = 0; u < 4; ++u) R[(row + 4 * u) * DLD + 16 * jb + col] = r[u];
    }
    __syncthreads();
    // tiles (ib, jb), ib != kb: updates for jb != kb, the new pivot column for
    // jb == kb; all reads of the old pivot column precede the writes
    double nv[3][4];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int tt = wave + 4 * s, ib = tt / 4 + (tt / 4 >= kb), jb = tt % 4;
      const dbl4c p = tile16([&](int m, int k) { return M[(16 * ib + m) * DLD + K0 + k]; },
                             [&](int k, int n) {
                               return jb == kb ? M[(K0 + k) * DLD + K0 + n] : R[k * DLD + 16 * jb + n];
                             });
#pragma unroll
      for (int u = 0; u < 4; ++u)
        nv[s][u] = jb == kb ? -p[u] : M[(16 * ib + row + 4 * u) * DLD + 16 * jb + col] - p[u];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int tt = wave + 4 * s, ib = tt / 4 + (tt / 4 >= kb), jb = tt % 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) M[(16 * ib + row + 4 * u) * DLD + 16 * jb + col] = nv[s][u];
    }
    // the new pivot rows
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q, r = e >> 6, j = e & 63;
      if ((j >> 4) != kb) M[(K0 + r) * DLD + j] = R[r * DLD + j];
    }
    __syncthreads();
  }
  if (t == 0 && bad) atomicOr(flags, 32);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = (t >> 6) + 4 * q, j = t & 63;
    if (i < kn && j < kn) A[(long long)i * nf + j] = M[i * DLD + j];
  }
}

// 64 x 64 x kn product on a 16 x 16 thread grid, 4 x 4 outputs per thread:
// acc[a][b] = sum_q X[q][tr + 16a] Y[q][tc + 16b]  (X stored transposed)
template <int LX>
__device__ inline void tile_product(const double (*X)[LX], const double (*Y)[GJB], int kn, double (&acc)[4][4]) {
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int q = 0; q < kn; ++q) {
    double x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = X[q][tr + 16 * a];
#pragma unroll
    for (int b = 0; b < 4; ++b) y[b] = Y[q][tc + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
  }
}

// grid (column tiles, fronts)
__global__ __launch_bounds__(256) void k_lv_panel(const NDNodeH* __restrict__ nodes, const int* __restrict__ lvl,
                                                  double* __restrict__ F, int k0, double* __restrict__ Cp) {
  __shared__ double Pt[GJB][GJB + 1];  // Pt[q][a] = P[a][q]
  __shared__ double As[GJB][GJB];  // As[q][b] = F[k0 + q][j0 + b]
  const NDNodeH d = nodes[lvl[blockIdx.y]];
  const int nf = d.ns + d.nb, j0 = blockIdx.x * GJB;
  if (k0 >= d.ns || j0 >= nf) return;
  const int kn = min(GJB, d.ns - k0);
  double* A = F + d.foff;
  const int t = threadIdx.x;
  double* cp = Cp + d.cp_off;
  const bool any = j0 != k0 || kn < GJB;  // the tile holds columns outside K
  // every load first, from clamped addresses (values outside the ranges are
  // not used), so that the 48 loads of a thread are in flight together:
  // the pivot-column block of the tile's rows (for Cp), F[K][K], the tile's
  // pivot rows
  double vc[16], vp[16], va[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = t + 256 * m, r = idx >> 6, q = idx & 63, i = j0 + r;
    vc[m] = A[(long long)(i < nf ? i : 0) * nf + k0 + (q < kn ? q : 0)];
  }
  if (any) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int idx = t + 256 * m, a = idx >> 6, b = idx & 63, j = j0 + b;
      const long long row = (long long)(k0 + (a < kn ? a : 0)) * nf;
      vp[m] = A[row + k0 + (b < kn ? b : 0)];
      va[m] = A[row + (j < nf ? j : 0)];
    }
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = t + 256 * m, r = idx >> 6, q = idx & 63, i = j0 + r;
    if (i < nf && q < kn && (i < k0 || i >= k0 + kn)) cp[(long long)i * GJB + q] = vc[m];
  }
  if (!any) return;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = t + 256 * m, a = idx >> 6, b = idx & 63, j = j0 + b;
    Pt[b][a] = (a < kn && b < kn) ? vp[m] : 0.0;
    As[a][b] = (a < kn && j < nf) ? va[m] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
  tile_product(Pt, As, kn, acc);
  const int tr = t >> 4, tc = t & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = tr + 16 * a, j = j0 + tc + 16 * b;
      if (r < kn && j < nf && (j < k0 || j >= k0 + kn)) A[(long long)(k0 + r) * nf + j] = acc[a][b];
    }
}

// grid (column tiles, row tiles, fronts)
__global__ __launch_bounds__(256) void k_lv_update(const NDNodeH* __restrict__ nodes, const int* __restrict__ lvl,
                                                   double* __restrict__ F, int k0, const double* __restrict__ Cp) {
  __shared__ double Ct[GJB][GJB + 1];  // Ct[q][r] = Cp[i0 + r][q]
  __shared__ double Rs[GJB][GJB];  // Rs[q][b] = F[k0 + q][j0 + b]
  const NDNodeH d = nodes[lvl[blockIdx.z]];
  const int nf = d.ns + d.nb, j0 = blockIdx.x * GJB, i0 = blockIdx.y * GJB;
  if (k0 >= d.ns || j0 >= nf || i0 >= nf) return;
  const int kn = min(GJB, d.ns - k0);
  if (i0 == k0 && kn == GJB) return;  // pivot rows only
  double* A = F + d.foff;
  const double* cp = Cp + d.cp_off;
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  // every load first, from clamped addresses: Cp and the pivot rows for the
  // product, and the thread's 16 old entries, which stay in flight during it
  double vct[16], vrs[16], old[4][4];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = t + 256 * m, r = idx >> 6, q = idx & 63, i = i0 + r, j = j0 + q;
    vct[m] = cp[(long long)(i < nf ? i : 0) * GJB + (q < kn ? q : 0)];
    vrs[m] = A[(long long)(k0 + (r < kn ? r : 0)) * nf + (j < nf ? j : 0)];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
      old[a][b] = A[(long long)(i < nf ? i : 0) * nf + (j < nf ? j : 0)];
    }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = t + 256 * m, r = idx >> 6, q = idx & 63, i = i0 + r, j = j0 + q;
    Ct[q][r] = (i < nf && q < kn && (i < k0 || i >= k0 + kn)) ? vct[m] : 0.0;
    Rs[r][q] = (r < kn && j < nf) ? vrs[m] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
  tile_product(Ct, Rs, kn, acc);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
      if (i >= nf || j >= nf || (i >= k0 && i < k0 + kn)) continue;
      A[(long long)i * nf + j] = (j >= k0 && j < k0 + kn) ? -acc[a][b] : old[a][b] - acc[a][b];
    }
}

// Same update as k_lv_update, one workgroup per 64-row strip of a front: the
// strip's old pivot-column block is staged once and the column tiles are
// streamed, so every entry of the front is read and written once per pivot
// block (the pivot rows come from L2).  grid (row strips, fronts).
__global__ __launch_bounds__(256) void k_lv_update_rows(const NDNodeH* __restrict__ nodes,
                                                        const int* __restrict__ lvl, double* __restrict__ F, int k0,
                                                        const double* __restrict__ Cp) {
  __shared__ double Ct[GJB][GJB + 1];  // Ct[q][r] = Cp[i0 + r][q]
  __shared__ double Rs[GJB][GJB];      // Rs[q][b] = F[k0 + q][j0 + b]
  const NDNodeH d = nodes[lvl[blockIdx.y]];
  const int nf = d.ns + d.nb, i0 = blockIdx.x * GJB;
  if (k0 >= d.ns || i0 >= nf) return;
  const int kn = min(GJB, d.ns - k0);
  if (i0 == k0 && kn == GJB) return;  // pivot rows only
  double* A = F + d.foff;
  const double* cp = Cp + d.cp_off;
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  // loads from clamped addresses, all of a tile's in flight together; the
  // next tile's pivot rows and old entries are requested before the current
  // tile's product
  double vrs[16], old[4][4];
  auto load_tile = [&](int j0) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int idx = t + 256 * m, r = idx >> 6, q = idx & 63, j = j0 + q;
      vrs[m] = A[(long long)(k0 + (r < kn ? r : 0)) * nf + (j < nf ? j : 0)];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
        old[a][b] = A[(long long)(i < nf ? i : 0) * nf + (j < nf ? j : 0)];
      }
  };
  {
    double vct[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int idx = t + 256 * m, r = idx >> 6, q = idx & 63, i = i0 + r;
      vct[m] = cp[(long long)(i < nf ? i : 0) * GJB + (q < kn ? q : 0)];
    }
    load_tile(0);
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int idx = t + 256 * m, r = idx >> 6, q = idx & 63, i = i0 + r;
      Ct[q][r] = (i < nf && q < kn && (i < k0 || i >= k0 + kn)) ? vct[m] : 0.0;
    }
  }
  for (int j0 = 0; j0 < nf; j0 += GJB) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int idx = t + 256 * m, r = idx >> 6, q = idx & 63, j = j0 + q;
      Rs[r][q] = (r < kn && j < nf) ? vrs[m] : 0.0;
    }
    double cur[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) cur[a][b] = old[a][b];
    __syncthreads();
    if (j0 + GJB < nf) load_tile(j0 + GJB);
    double acc[4][4];
    tile_product(Ct, Rs, kn, acc);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
        if (i >= nf || j >= nf || (i >= k0 && i < k0 + kn)) continue;
        A[(long long)i * nf + j] = (j >= k0 && j < k0 + kn) ? -acc[a][b] : cur[a][b] - acc[a][b];
      }
    __syncthreads();
  }
}

hipError_t launch_coarse_assemble(Ctx* c) {
  const CoarseLayout& co = c->co;
  hipLaunchKernelGGL(k_fill, dim3(2048), dim3(256), 0, c->stream, c->d_coarse, co.nd_front_total, 0.0);
  int nent = (int)co.dest.size();
  hipLaunchKernelGGL(k_coarse_entries, dim3((nent + 255) / 256), dim3(256), 0, c->stream, c->d_ScLoc, c->d_cstart,
                     c->d_contrib, c->d_dest, c->d_coarse, nent);
  return hipGetLastError();
}

// Copy the M^T rows of the fronts of the fused subtrees into their packed
// forward blocks (once per factorization).  One workgroup per node.
__global__ __launch_bounds__(256) void k_fused_pack(const FusedPack* __restrict__ pk, const double* __restrict__ F,
                                                    double* __restrict__ blk) {
  const FusedPack q = pk[blockIdx.x];
  const int nf = q.ns + q.nb, n = q.ns * q.nb;
  for (int i = threadIdx.x; i < n; i += 256) {
    const int k = i / q.nb, r = i - k * q.nb;
    blk[q.fdst + i] = F[q.foff + (long long)k * nf + q.ns + r];
  }
}

hipError_t launch_coarse_factor(Ctx* c) {
  const CoarseLayout& co = c->co;
  for (int l = (int)co.nd_levels.size() - 1; l >= 0; --l) {
    const int n0 = co.lvl_off[l], nn = co.lvl_off[l + 1] - n0;
    const int* lvl = c->d_lvl_nodes + n0;
    int nbmax = 0, nfmax = 0, nsmax = 0;
    for (int n : co.nd_levels[l]) {
      const NDNodeH& d = co.nd_nodes[n];
      nfmax = std::max(nfmax, d.ns + d.nb);
      nsmax = std::max(nsmax, d.ns);
      for (int s = 0; s < 2; ++s)
        if (d.child[s] >= 0) nbmax = std::max(nbmax, co.nd_nodes[d.child[s]].nb);
    }
    if (nfmax <= 72) {
      hipLaunchKernelGGL((k_front_lds<72, 256>), dim3(nn), dim3(256), 0, c->stream, c->d_nd_nodes, lvl, c->d_nd_cmap,
                         c->d_coarse, c->d_flags);
      continue;
    }
    if (nfmax <= ND_LDS_NF) {
      hipLaunchKernelGGL((k_front_lds<ND_LDS_NF, 512>), dim3(nn), dim3(512), 0, c->stream, c->d_nd_nodes, lvl,
                         c->d_nd_cmap, c->d_coarse, c->d_flags);
      continue;
    }
    if (nbmax > 0)
      for (int s = 0; s < 2; ++s) {
        const dim3 g(nn, (nbmax + 15) / 16);
#define EXA(kc) hipLaunchKernelGGL(k_extend_add<kc>, g, dim3(256), 0, c->stream, c->d_nd_nodes, lvl, c->d_nd_cmap, c->d_coarse, s)
        if (nbmax <= 128) EXA(2);
        else if (nbmax <= 256) EXA(4);
        else if (nbmax <= 512) EXA(8);
        else if (nbmax <= 1024) EXA(16);
        else EXA(0);
#undef EXA
      }
    const int nt = (nfmax + GJB - 1) / GJB;
    for (int k0 = 0; k0 < nsmax; k0 += GJB) {
      hipLaunchKernelGGL(k_lv_diag, dim3(nn), dim3(256), 0, c->stream, c->d_nd_nodes, lvl, c->d_coarse, k0,
                         c->d_flags);
      hipLaunchKernelGGL(k_lv_panel, dim3(nt, nn), dim3(256), 0, c->stream, c->d_nd_nodes, lvl, c->d_coarse, k0,
                         c->d_gjC);
      if (nn >= 32)  // enough fronts to fill the chip with row strips
        hipLaunchKernelGGL(k_lv_update_rows, dim3(nt, nn), dim3(256), 0, c->stream, c->d_nd_nodes, lvl,
                           c->d_coarse, k0, c->d_gjC);
      else
        hipLaunchKernelGGL(k_lv_update, dim3(nt, nt, nn), dim3(256), 0, c->stream, c->d_nd_nodes, lvl, c->d_coarse,
                           k0, c->d_gjC);
    }
  }
  if (co.fused) {
    const hipError_t e = prepare_fused_sweeps(c);
    if (e != hipSuccess) return e;
  }
  if (co.fused && !co.f_pack.empty())
    hipLaunchKernelGGL(k_fused_pack, dim3((unsigned)co.f_pack.size()), dim3(256), 0, c->stream, c->d_f_pack,
                       c->d_coarse, c->d_f_blk);
  return hipGetLastError();
}

// Both sweeps read only the top ns rows of a swept front, [F_ss^-1 | M^T]
// (row-major, row stride nf); the lower rows are not needed once the parent
// has taken U.

// Sum over a child's parts of its up-vector entry at one front position, in
// part order, for the two children at once.  src = the index in `up` of part 0
// of each child's entry (-1: the child does not touch this position; part u
// is u * child_nb further).  pull_load requests the first CK parts of both
// children unconditionally (a position that is not needed reads up[0]), so
// that the loads of several positions can all be in flight before pull_sum
// adds them; pull_sum adds any further parts in a loop.
template <int CK>
struct Pulled {
  double t0[CK], t1[CK];
  int n0, n1;
};
template <int CK>
__device__ __forceinline__ Pulled<CK> pull_load(const NDItem& d, const double* __restrict__ up, int2 src) {
  Pulled<CK> p;
  p.n0 = src.x >= 0 ? d.child_kparts[0] : 0;
  p.n1 = src.y >= 0 ? d.child_kparts[1] : 0;
#pragma unroll
  for (int u = 0; u < CK; ++u) p.t0[u] = up[u < p.n0 ? src.x + u * d.child_nb[0] : 0];
#pragma unroll
  for (int u = 0; u < CK; ++u) p.t1[u] = up[u < p.n1 ? src.y + u * d.child_nb[1] : 0];
  return p;
}
template <int CK>
__device__ __forceinline__ void pull_sum(const NDItem& d, const double* __restrict__ up, int2 src,
                                         const Pulled<CK>& p, double& c0, double& c1) {
  c0 = 0.0;
  c1 = 0.0;
#pragma unroll
  for (int u = 0; u < CK; ++u) c0 += u < p.n0 ? p.t0[u] : 0.0;
#pragma unroll
  for (int u = 0; u < CK; ++u) c1 += u < p.n1 ? p.t1[u] : 0.0;
  for (int kp = CK; kp < p.n0; ++kp) c0 += up[src.x + kp * d.child_nb[0]];
  for (int kp = CK; kp < p.n1; ++kp) c1 += up[src.y + kp * d.child_nb[1]];
}

// Forward item (node, boundary columns [r0, r0 + 64), own-row part kp = rows
// [kb, ke), ke - kb <= 64):
//   w_k = b_k + (children's contributions to own row k),          k in [kb, ke)
//   w_b[r] = children's contributions to boundary position r,       (part 0)
//   part_kp[r] = [kp == 0] w_b[r] - sum_{k in [kb, ke)} w_k M^T[k][r]
// The node's up vector is the sum of its parts, added in order by the parent;
// the children's contributions are pulled through the node's pull map, so an
// item gathers only the 64 rows and 64 columns it uses.  Lane = column r
// (coalesced rows of M^T), wave wv takes rows kb + wv + 4u, u < 16, all
// requested before the right-hand side is gathered; the four wave partials
// are added in a fixed order.  The items of column block 0 store b_eff of
// their rows for the backward sweep.
template <bool MC>
__global__ __launch_bounds__(256) void k_nd_fwd(const NDItem* __restrict__ items, const int2* __restrict__ fsrc,
                                                const double* __restrict__ F, const double* __restrict__ b,
                                                double* __restrict__ up, double* __restrict__ beff, SweepVecs sv) {
  if (sv.mask == 0u) return;
  const int k0 = __builtin_ctz(sv.mask);  // the first load case; the M^T rows serve every case
  __shared__ double w[128];  // [0, 64): w on rows kb.., [64, 128): w_b on columns r0..
  __shared__ double pr[4][64];
  const NDItem d = items[blockIdx.x];
  const int nf = d.ns + d.nb, t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6, r = d.first + lane;
  const int kb = d.kpart * ND_KPART, ke = min(d.ns, kb + ND_KPART);
  const bool col_ok = r < d.nb;
  // front position of threads t < 128: own row kb + t, or boundary column
  // r0 + t - 64; positions that are not needed read index 0 and are discarded
  const bool own = t < 64;
  const bool ok = t < 128 && (own ? kb + t < ke : (d.kpart == 0 && d.first + (t - 64) < d.nb));
  const int j = ok ? (own ? kb + t : d.ns + d.first + (t - 64)) : 0;
  const int jb = ok && own ? d.own_off + j : 0;
  // the item's gather sources (at a position known before the item itself)
  // and b ahead of M^T (the counter is in order)
  const int2 srcl = fsrc[(long long)blockIdx.x * 128 + (t < 128 ? t : 0)];
  const double bj0 = b[k0 * sv.v + jb];
  __builtin_amdgcn_sched_barrier(0);
  // unconditional loads of M^T: rows past ke read row 0 and meet zeros of w,
  // columns past nb read F[0] and are not stored (factor entries are finite)
  const double* col = col_ok ? F + d.foff + d.ns + r : F;
  double a[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int k = kb + wv + 4 * u;
    a[u] = col[col_ok && k < ke ? (long long)k * nf : 0];
  }
  for (int k = k0; k < (MC ? sv.nr : k0 + 1); ++k) {
    if (MC && !((sv.mask >> k) & 1u)) continue;
    double* __restrict__ upk = up + k * sv.up;
    if (t < 128) {
      double v = own ? (k == k0 ? bj0 : b[k * sv.v + jb]) : 0.0;
      {
        double c0, c1;
        const int2 src = ok ? srcl : make_int2(-1, -1);
        pull_sum<8>(d, upk, src, pull_load<8>(d, upk, src), c0, c1);
        v += c0;
        v += c1;
      }
      v = ok ? v : 0.0;
      if (ok && own && d.first == 0) beff[k * sv.beff + d.own_off + j] = v;
      w[t] = v;
    }
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) s += a[u] * w[wv + 4 * u];
    pr[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && col_ok) {
      const double tot = ((pr[0][lane] + pr[1][lane]) + pr[2][lane]) + pr[3][lane];
      upk[d.up_off + d.kpart * d.nb + r] = (d.kpart == 0 ? w[64 + lane] : 0.0) - tot;
    }
    __syncthreads();  // w and pr are rewritten for the next case
  }
}

// Backward item (node, own rows [k0, k0 + 4Q)): rows of
// g_s = [F_ss^-1 | M^T] [b_eff; -g_b].  Wave wv takes rows k0 + wv + 4q;
// lanes run along a row in passes of NCH chunks of 64 columns, every load of
// a pass requested before its first use (the first pass before the vector is
// gathered); a butterfly sums each row.  LDS: nf doubles rounded up to a
// multiple of 1024.
template <int Q, int NCH, bool MC>
__global__ __launch_bounds__(256) void k_nd_bwd(const NDItem* __restrict__ items, const int* __restrict__ bnd,
                                                const double* __restrict__ F, const double* __restrict__ beff,
                                                double* __restrict__ x, SweepVecs sv) {
  extern __shared__ double sh[];
  const NDItem d = items[blockIdx.x];
  if (d.ns == 0 || sv.mask == 0u) return;  // no own rows (the whole workgroup)
  const int nf = d.ns + d.nb, t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  // boundary indices of the first 1024 front positions (four per thread)
  int g0[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int j = t + 256 * m;
    g0[m] = bnd[(j >= d.ns && j < nf) ? d.bnd_off + j - d.ns : 0];
  }
  // keep the index loads ahead of the row loads (the counter is in order)
  __builtin_amdgcn_sched_barrier(0);
  const double* rows[Q];
  bool ok[Q];
  double a[Q][NCH];
  // row loads are unconditional, so the compiler counts them exactly and the
  // gather waits for the indices alone: columns past nf read the row's first
  // entry and meet zeros of the padded vector, rows past ns read the front's
  // first row and are not stored (factor entries are finite)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = d.first + wv + 4 * q;
    ok[q] = k < d.ns;
    rows[q] = F + d.foff + (long long)(ok[q] ? k : 0) * nf;
  }
  auto load_pass = [&](int c0) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int j = c0 + lane + 64 * c;
        a[q][c] = rows[q][j < nf ? j : 0];
      }
  };
  load_pass(0);
  // the first pass of rows stays in registers for every load case in the mask
  // (fronts wider than one pass reload it, from the cache, for the next case)
  const bool multi = nf > 64 * NCH;
  bool first = true;
  for (int k = 0; k < (MC ? sv.nr : 1); ++k) {
    if (MC && !((sv.mask >> k) & 1u)) continue;
    const double* __restrict__ bk = beff + k * sv.beff;
    double* __restrict__ xk = x + k * sv.v;
    if (!first) {
      __syncthreads();  // the previous case's reads of sh are done
      if (multi) load_pass(0);
    }
    first = false;
    // [b_eff; -x_b] into LDS: one load per position through a selected
    // address, every value stored (the LDS vector is padded to a multiple of
    // 1024); the first 1024 positions with the indices read above
    auto gather = [&](int j0, const int (&g)[4]) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int j = j0 + t + 256 * m;
        const bool is_b = j >= d.ns && j < nf, is_s = j < d.ns;
        const double l = *(is_b ? xk + g[m] : bk + (is_s ? d.own_off + j : 0));
        sh[j] = is_b ? -l : (is_s ? l : 0.0);
      }
    };
    gather(0, g0);
    for (int j0 = 1024; j0 < nf; j0 += 1024) {
      int g[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int j = j0 + t + 256 * m;
        g[m] = bnd[(j >= d.ns && j < nf) ? d.bnd_off + j - d.ns : 0];
      }
      gather(j0, g);
    }
    __syncthreads();
    double s[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] = 0.0;
    for (int c0 = 0;;) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double vj = sh[c0 + lane + 64 * c];
#pragma unroll
        for (int q = 0; q < Q; ++q) s[q] += a[q][c] * vj;
      }
      c0 += 64 * NCH;
      if (c0 >= nf) break;
      load_pass(c0);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      double v = s[q];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0 && ok[q]) xk[d.own_off + d.first + wv + 4 * q] = v;
    }
  }
}

// Lane l's copy of a double held by lane `src` (wave-uniform src), through
// two scalar reads.
__device__ __forceinline__ double read_lane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Forward item with at most R own rows, taken by one wave: the item of
// k_nd_fwd.  Lane l pulls front position kb + l (own row) and boundary
// column r0 + l, reads the R rows of M^T in its column, and takes w_k from
// lane k - kb.
template <int R, int CK, bool MC>
__device__ __forceinline__ void fwd_task(const NDItem& d, const int2* __restrict__ fsrc,
                                         const double* __restrict__ F, const double* __restrict__ b,
                                         double* __restrict__ up, double* __restrict__ beff, const SweepVecs& sv) {
  const int lane = threadIdx.x & 63, nf = d.ns + d.nb, r = d.first + lane;
  const int kb = d.kpart * ND_KPART, ke = min(d.ns, kb + R);
  const bool col_ok = r < d.nb;
  const bool ok1 = kb + lane < ke, ok2 = d.kpart == 0 && col_ok;
  const int j1 = ok1 ? kb + lane : 0, j2 = ok2 ? d.ns + r : 0;
  const bool has_ch = d.pull_off >= 0;
  const int2 s1 = fsrc[lane];
  const int2 s2 = fsrc[64 + lane];
  const int k0 = __builtin_ctz(sv.mask);
  const double b10 = b[k0 * sv.v + (ok1 ? d.own_off + j1 : 0)];
  __builtin_amdgcn_sched_barrier(0);  // indices ahead of M^T (the counter is in order)
  // rows past ke read row 0 and meet w = 0; columns past nb are not stored
  const double* col = col_ok ? F + d.foff + d.ns + r : F;
  double a[R];
#pragma unroll
  for (int u = 0; u < R; ++u) a[u] = col[col_ok && kb + u < ke ? (long long)(kb + u) * nf : 0];
  // the rows of M^T stay in registers for every load case in the mask
  for (int k = k0; k < (MC ? sv.nr : k0 + 1); ++k) {
    if (MC && !((sv.mask >> k) & 1u)) continue;
    double* __restrict__ upk = up + k * sv.up;
    double w1 = k == k0 ? b10 : b[k * sv.v + (ok1 ? d.own_off + j1 : 0)], w2 = 0.0;
    if (has_ch) {
      double c0, c1, e0, e1;
      const int2 p1 = ok1 ? s1 : make_int2(-1, -1), p2 = ok2 ? s2 : make_int2(-1, -1);
      const Pulled<CK> l1 = pull_load<CK>(d, upk, p1);
      const Pulled<CK> l2 = pull_load<CK>(d, upk, p2);
      pull_sum<CK>(d, upk, p1, l1, c0, c1);
      pull_sum<CK>(d, upk, p2, l2, e0, e1);
      w1 += c0;
      w1 += c1;
      w2 += e0;
      w2 += e1;
    }
    w1 = ok1 ? w1 : 0.0;
    if (ok1 && d.first == 0) beff[k * sv.beff + d.own_off + j1] = w1;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) acc += a[u] * read_lane(w1, u);
    if (col_ok) upk[d.up_off + d.kpart * d.nb + r] = (d.kpart == 0 ? w2 : 0.0) - acc;
  }
}

// Backward item of 16 own rows [k0, k0 + 16) taken by one wave: rows of
// g_s = [F_ss^-1 | M^T] [b_eff; -g_b] with nf <= 64 NCH.  Lane l owns columns
// l + 64c and gathers their vector entries itself (no LDS); a reduce-scatter
// over the lanes leaves row 8 b5 + 4 b4 + 2 b3 + b2 (bits of the lane id) in
// the lanes with b1 = b0 = 0.
static_assert(ND_BW_ROWS == 16, "bwd_task takes items of 16 rows");
template <int NCH, bool MC>
__device__ __forceinline__ void bwd_task(const NDItem& d, const int* __restrict__ bnd, const double* __restrict__ F,
                                         const double* __restrict__ beff, double* __restrict__ x, const SweepVecs& sv) {
  if (d.ns == 0) return;
  const int lane = threadIdx.x & 63, nf = d.ns + d.nb;
  int g[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j = lane + 64 * c;
    g[c] = bnd[(j >= d.ns && j < nf) ? d.bnd_off + j - d.ns : 0];
  }
  __builtin_amdgcn_sched_barrier(0);  // indices ahead of the rows (the counter is in order)
  // rows past ns read row 0 and are not stored; columns past nf meet v = 0
  double a[16][NCH];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = d.first + q;
    const double* row = F + d.foff + (long long)(k < d.ns ? k : 0) * nf;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int j = lane + 64 * c;
      a[q][c] = row[j < nf ? j : 0];
    }
  }
  // the rows stay in registers for every load case in the mask
  for (int k = 0; k < (MC ? sv.nr : 1); ++k) {
  if (MC && !((sv.mask >> k) & 1u)) continue;
  const double* __restrict__ bk = beff + k * sv.beff;
  double* __restrict__ xk = x + k * sv.v;
  double v[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j = lane + 64 * c;
    const bool is_b = j >= d.ns && j < nf, is_s = j < d.ns;
    const double l = *(is_b ? xk + g[c] : bk + (is_s ? d.own_off + j : 0));
    v[c] = is_b ? -l : (is_s ? l : 0.0);
  }
  double s[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    s[q] = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) s[q] += a[q][c] * v[c];
  }
  // reduce-scatter: at each step a lane keeps the half of its rows selected by
  // one bit of its id and adds the partner's copy of that half
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
  double t8[8], t4[4], t2[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double keep = b5 ? s[8 + i] : s[i], send = b5 ? s[i] : s[8 + i];
    t8[i] = keep + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double keep = b4 ? t8[4 + i] : t8[i], send = b4 ? t8[i] : t8[4 + i];
    t4[i] = keep + __shfl_xor(send, 16);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = b3 ? t4[2 + i] : t4[i], send = b3 ? t4[i] : t4[2 + i];
    t2[i] = keep + __shfl_xor(send, 8);
  }
  double t1;
  {
    const double keep = b2 ? t2[1] : t2[0], send = b2 ? t2[0] : t2[1];
    t1 = keep + __shfl_xor(send, 4);
  }
  t1 += __shfl_xor(t1, 2);
  t1 += __shfl_xor(t1, 1);
  const int q = (b5 ? 8 : 0) + (b4 ? 4 : 0) + (b3 ? 2 : 0) + (b2 ? 1 : 0);
  if ((lane & 3) == 0 && d.first + q < d.ns) xk[d.own_off + d.first + q] = t1;
  }
}

// Items of the lower tree levels (many small fronts): one per wave, four
// per workgroup.
template <int R, int CK, bool MC>
__global__ __launch_bounds__(256) void k_nd_fwd_w(const NDItem* __restrict__ items, int nitems,
                                                  const int2* __restrict__ fsrc, const double* __restrict__ F,
                                                  const double* __restrict__ b, double* __restrict__ up,
                                                  double* __restrict__ beff, SweepVecs sv) {
  if (sv.mask == 0u) return;
  const int it = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (all load cases)
  if (it < nitems) fwd_task<R, CK, MC>(items[it], fsrc + (long long)it * 128, F, b, up, beff, sv);
}
template <int NCH, bool MC>
__global__ __launch_bounds__(256) void k_nd_bwd_w(const NDItem* __restrict__ items, int nitems,
                                                  const int* __restrict__ bnd, const double* __restrict__ F,
                                                  const double* __restrict__ beff, double* __restrict__ x, SweepVecs sv) {
  const int it = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (all load cases)
  if (it < nitems) bwd_task<NCH, MC>(items[it], bnd, F, beff, x, sv);
}

// The bottom levels of the tree in one launch per sweep: workgroup = one
// subtree, processed in nst stages (forward: deepest level first; backward:
// the subtree root first), the stage's items taken by the four waves in turn.
// The items of a stage read what the previous stages of the same workgroup
// wrote to global memory (up vectors, solution entries): the barrier between
// stages orders them at workgroup scope.  stage_off[(sub) (nst + 1) + s] is
// the first item of stage s of subtree `sub`.
template <int R, int CK, bool MC>
__global__ __launch_bounds__(256) void k_nd_fwd_sub(const NDItem* __restrict__ items,
                                                    const int* __restrict__ stage_off, int nst,
                                                    const int2* __restrict__ fsrc, const double* __restrict__ F,
                                                    const double* __restrict__ b, double* __restrict__ up,
                                                    double* __restrict__ beff, SweepVecs sv) {
  if (sv.mask == 0u) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int* so = stage_off + (long long)blockIdx.x * (nst + 1);  // (all load cases)
  for (int st = 0; st < nst; ++st) {
    for (int it = so[st] + wv; it < so[st + 1]; it += 4)
      fwd_task<R, CK, MC>(items[it], fsrc + (long long)it * 128, F, b, up, beff, sv);
    __syncthreads();
  }
}
template <int NCH, bool MC>
__global__ __launch_bounds__(256) void k_nd_bwd_sub(const NDItem* __restrict__ items,
                                                    const int* __restrict__ stage_off, int nst,
                                                    const int* __restrict__ bnd, const double* __restrict__ F,
                                                    const double* __restrict__ beff, double* __restrict__ x, SweepVecs sv) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int* so = stage_off + (long long)blockIdx.x * (nst + 1);  // (all load cases)
  for (int st = 0; st < nst; ++st) {
    for (int it = so[st] + wv; it < so[st + 1]; it += 4) bwd_task<NCH, MC>(items[it], bnd, F, beff, x, sv);
    __syncthreads();
  }
}

// Fused forward sweep of the bottom ND_FUSED_LEVELS levels: one workgroup per
// subtree.  Everything the subtree reads (its packed M^T rows, its vector
// entry program, its node table, its own right-hand side) is requested at the
// start with every load in flight and staged in LDS; the levels then follow
// one another through LDS with workgroup barriers only, so a subtree costs
// about one round trip to memory instead of a few per level.  The subtree
// root's up vector and the b_eff of every own row go to global memory.
// The node of depth range [n0, n1) (at most ND_FUSED_STAGE_NODES nodes) whose
// (node, column) pairs (first pair in pair0) contain pair idx: the reads of
// the table are unconditional (clamped), so they are issued together.
__device__ __forceinline__ int fused_node_of(const FusedNode* nd, int n0, int n1, int idx) {
  int i = n0;
#pragma unroll
  for (int u = 1; u < ND_FUSED_STAGE_NODES; ++u) {
    const int cidx = n0 + u < n1 ? n0 + u : n0;
    const int first = nd[cidx].pair0;
    if (n0 + u < n1 && first <= idx) i = n0 + u;
  }
  return i;
}

__device__ __forceinline__ void fused_levels(const FusedSub& S, const FusedNode* nd, const short4 (&e)[ND_FUSED_ENT],
                                             int e0, const double* sh, double* vec, const double* bvs,
                                             double* __restrict__ up, double* __restrict__ beff);
template <bool MC>
__global__ __launch_bounds__(ND_FUSED_THREADS) void k_nd_fwd_fused(const FusedSub* __restrict__ subs,
                                                                   const FusedNode* __restrict__ nodes,
                                                                   const short4* __restrict__ went,
                                                                   const double* __restrict__ blk,
                                                                   const double* __restrict__ b,
                                                                   double* __restrict__ up, double* __restrict__ beff, SweepVecs sv) {
  // one workgroup per subtree for all load cases: the subtree's data is staged
  // once, the levels run once per case in the mask
  if (sv.mask == 0u) return;
  const int k0 = __builtin_ctz(sv.mask);
  extern __shared__ double2 sh2[];  // 16-byte aligned for the block stores
  double* sh = reinterpret_cast<double*>(sh2);
  __shared__ FusedNode nd[16];
  const int t = threadIdx.x;
  const FusedSub S = subs[blockIdx.x];
  const int nnode = S.stage_node[ND_FUSED_LEVELS];
  // every independent load first: the block (16-byte loads from clamped
  // positions), the entry program, the node table, the own right-hand side
  const double2* src = reinterpret_cast<const double2*>(blk + S.fwd_off);
  const int nb2 = S.fwd_n >> 1;
  double2 a[ND_FUSED_LOADS];
#pragma unroll
  for (int u = 0; u < ND_FUSED_LOADS; ++u) {
    const int i = t + ND_FUSED_THREADS * u;
    a[u] = src[i < nb2 ? i : 0];
  }
  const int e0 = S.went[0], e1 = S.went[ND_FUSED_LEVELS];
  short4 e[ND_FUSED_ENT];
#pragma unroll
  for (int u = 0; u < ND_FUSED_ENT; ++u) {
    const int i = e0 + t + ND_FUSED_THREADS * u;
    e[u] = went[i < e1 ? i : e0];
  }
  const FusedNode fn = nodes[S.node0 + (t < nnode ? t : 0)];
  const double bv = b[k0 * sv.v + S.own_off + (t < S.own_n ? t : 0)];
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the first store
  // unconditional stores (a lane past the end stores what it read from the
  // clamped position, the same value as the owner of that position), so that
  // no load is moved behind a branch and all of them stay in flight together
  double2* sb = sh2;
#pragma unroll
  for (int u = 0; u < ND_FUSED_LOADS; ++u) {
    const int i = t + ND_FUSED_THREADS * u;
    sb[i < nb2 ? i : 0] = a[u];
  }
  double* vec = sh + S.fwd_n;
  double* bvs = vec + S.vec_n;
  nd[t < nnode ? t : 0] = fn;
  bvs[t < S.own_n ? t : 0] = bv;
  for (int k = k0; k < (MC ? sv.nr : k0 + 1); ++k) {
    if (MC && !((sv.mask >> k) & 1u)) continue;
    double* upk = up + k * sv.up;
    double* beffk = beff + k * sv.beff;
    if (k != k0) {  // the previous case's last level ended with a barrier
      const double bk = b[k * sv.v + S.own_off + (t < S.own_n ? t : 0)];
      bvs[t < S.own_n ? t : 0] = bk;
    }
    __syncthreads();
    fused_levels(S, nd, e, e0, sh, vec, bvs, upk, beffk);
  }
}

// The levels of one fused forward sweep for one load case (the subtree's
// M^T, node table and entry program staged, the case's own right-hand side in
// bvs): see k_nd_fwd_fused.
__device__ __forceinline__ void fused_levels(const FusedSub& S, const FusedNode* nd, const short4 (&e)[ND_FUSED_ENT],
                                             int e0, const double* sh, double* vec, const double* bvs,
                                             double* __restrict__ up, double* __restrict__ beff) {
  const int t = threadIdx.x;
  for (int d = ND_FUSED_LEVELS - 1; d >= 0; --d) {
    // w of every front position of the level's nodes: own right-hand side plus
    // the children's up vectors (b_eff of the own rows is kept for the
    // backward sweep)
    // (the LDS reads of the thread's entries are unconditional, from clamped
    // positions, so they are issued together; unused values are dropped)
    double bw[ND_FUSED_ENT], c0[ND_FUSED_ENT], c1[ND_FUSED_ENT];
#pragma unroll
    for (int u = 0; u < ND_FUSED_ENT; ++u) {
      const short4 q = e[u];
      bw[u] = bvs[q.w >= 0 ? q.w : 0];
      c0[u] = vec[q.y >= 0 ? q.y : 0];
      c1[u] = vec[q.z >= 0 ? q.z : 0];
    }
#pragma unroll
    for (int u = 0; u < ND_FUSED_ENT; ++u) {
      const int i = e0 + t + ND_FUSED_THREADS * u;
      if (i >= S.went[d] && i < S.went[d + 1]) {
        const short4 q = e[u];
        double v = q.w >= 0 ? bw[u] : 0.0;
        if (q.y >= 0) v += c0[u];
        if (q.z >= 0) v += c1[u];
        vec[q.x] = v;
        if (q.w >= 0) beff[S.own_off + q.w] = v;
      }
    }
    __syncthreads();
    // up[r] = w_b[r] - sum_k M^T[k][r] w_k, one (node, column) per thread
    if (t < S.stage_pairs[d]) {
      const int i = fused_node_of(nd, S.stage_node[d], S.stage_node[d + 1], t);
      {
        const FusedNode q = nd[i];
        const int r = t - q.pair0;
        const double* mt = sh + q.mt + r;
        const double* w = vec + q.w;
        // eight terms per step, their LDS reads issued together (positions past
        // ns read row k again and are not added)
        double acc = 0.0;
        for (int k = 0; k < q.ns; k += 8) {
          double m[8], ww[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int kk = k + u < q.ns ? k + u : k;
            m[u] = mt[kk * q.nb];
            ww[u] = w[kk];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (k + u < q.ns) acc += m[u] * ww[u];
        }
        const double v = w[q.ns + r] - acc;
        if (q.gup >= 0) up[q.gup + r] = v;
        else vec[q.up + r] = v;
      }
    }
    __syncthreads();
  }
}

static size_t fused_lds_bytes(const CoarseLayout& co);

// LDS beyond the default dynamic limit for the fused sweep kernels
hipError_t prepare_fused_sweeps(Ctx* c) {
  if (!c->co.fused) return hipSuccess;
  const int lds = (int)fused_lds_bytes(c->co);
  const hipError_t e = hipFuncSetAttribute((const void*)k_nd_fwd_fused<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_nd_fwd_fused<true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

static size_t fused_lds_bytes(const CoarseLayout& co) {
  size_t m = 0;
  for (const FusedSub& S : co.f_subs) m = std::max(m, (size_t)S.fwd_n + S.vec_n + S.own_n);
  return m * sizeof(double);
}

template <int Q, bool MC>
static void launch_bwd(int nch, int ni, size_t lds, hipStream_t st, const NDItem* items, const int* bnd,
                       const double* F, const double* beff, double* x, SweepVecs sv) {
  const dim3 grid(ni);
  if (nch <= 2)
    hipLaunchKernelGGL((k_nd_bwd<Q, 2, MC>), grid, dim3(256), lds, st, items, bnd, F, beff, x, sv);
  else if (nch <= 4)
    hipLaunchKernelGGL((k_nd_bwd<Q, 4, MC>), grid, dim3(256), lds, st, items, bnd, F, beff, x, sv);
  else if (nch <= 8)
    hipLaunchKernelGGL((k_nd_bwd<Q, 8, MC>), grid, dim3(256), lds, st, items, bnd, F, beff, x, sv);
  else
    hipLaunchKernelGGL((k_nd_bwd<Q, 16, MC>), grid, dim3(256), lds, st, items, bnd, F, beff, x, sv);
}

// Levels with at least this many items take the one-item-per-wave kernels.
constexpr int ND_WAVE_ITEMS = 512;

template <int R, bool MC>
static void launch_fwd_w(int ck, int ni, hipStream_t st, const NDItem* items, const int2* fsrc,
                         const double* F, const double* b, double* up, double* beff, SweepVecs sv) {
  const dim3 grid((ni + 3) / 4);
  if (ck <= 1)
    hipLaunchKernelGGL((k_nd_fwd_w<R, 1, MC>), grid, dim3(256), 0, st, items, ni, fsrc, F, b, up, beff, sv);
  else if (ck <= 2)
    hipLaunchKernelGGL((k_nd_fwd_w<R, 2, MC>), grid, dim3(256), 0, st, items, ni, fsrc, F, b, up, beff, sv);
  else
    hipLaunchKernelGGL((k_nd_fwd_w<R, 8, MC>), grid, dim3(256), 0, st, items, ni, fsrc, F, b, up, beff, sv);
}

template <int R, bool MC>
static void launch_fwd_sub(const Ctx* c, const double* rhs, SweepVecs sv) {
  const CoarseLayout& co = c->co;
  const int ck = co.sub_child_kparts;
  const dim3 grid(co.sub_count);
  const int2* pull = c->d_sub_fw_src;
  if (ck <= 1)
    hipLaunchKernelGGL((k_nd_fwd_sub<R, 1, MC>), grid, dim3(256), 0, c->stream, c->d_sub_fw_items, c->d_sub_fw_off,
                       co.sub_nst, pull, c->d_coarse, rhs, c->d_up, c->d_beff, sv);
  else if (ck <= 2)
    hipLaunchKernelGGL((k_nd_fwd_sub<R, 2, MC>), grid, dim3(256), 0, c->stream, c->d_sub_fw_items, c->d_sub_fw_off,
                       co.sub_nst, pull, c->d_coarse, rhs, c->d_up, c->d_beff, sv);
  else
    hipLaunchKernelGGL((k_nd_fwd_sub<R, 8, MC>), grid, dim3(256), 0, c->stream, c->d_sub_fw_items, c->d_sub_fw_off,
                       co.sub_nst, pull, c->d_coarse, rhs, c->d_up, c->d_beff, sv);
}

// The sweeps of one coarse solve; MC: the kernels loop over the load cases
// of sv (every workgroup reads its factor rows once for all of them), else
// one case (the instances without the loop keep the single-case registers).
template <bool MC>
static hipError_t coarse_sweeps(Ctx* c, const double* rhs, double* x, hipEvent_t mid, const SweepVecs& sv) {
  const CoarseLayout& co = c->co;
  const int L = (int)co.nd_levels.size();
  // forward: the subtrees of the bottom levels, then the upper levels one launch each
  int top = co.sub_level;
  // (several load cases: the per-wave subtree kernel, whose M^T rows stay in
  // registers for every case; the fused kernel runs its levels case by case)
  if (co.fused && !MC) {
    top = co.fused_level;
    hipLaunchKernelGGL(k_nd_fwd_fused<MC>, dim3((unsigned)co.f_subs.size()), dim3(ND_FUSED_THREADS),
                       fused_lds_bytes(co), c->stream, c->d_f_subs, c->d_f_nodes, c->d_f_went, c->d_f_blk,
                       rhs, c->d_up, c->d_beff, sv);
  } else if (co.sub_level < L) {
    const int rows = co.sub_fw_rows;
    if (rows <= 16)
      launch_fwd_sub<16, MC>(c, rhs, sv);
    else if (rows <= 32)
      launch_fwd_sub<32, MC>(c, rhs, sv);
    else if (rows <= 48)
      launch_fwd_sub<48, MC>(c, rhs, sv);
    else
      launch_fwd_sub<64, MC>(c, rhs, sv);
  }
  for (int l = top - 1; l >= 0; --l) {
    const int i0 = co.fw_off[l], ni = co.fw_off[l + 1] - i0;
    if (ni == 0) continue;
    const NDItem* it = c->d_fw_items + i0;
    const int2* pull = c->d_fw_src + (long long)i0 * 128;
    const int rows = co.lvl_fw_rows[l], ck = co.lvl_child_kparts[l];
    if (ni >= ND_WAVE_ITEMS && rows <= 48) {
      if (rows <= 16)
        launch_fwd_w<16, MC>(ck, ni, c->stream, it, pull, c->d_coarse, rhs, c->d_up, c->d_beff, sv);
      else if (rows <= 32)
        launch_fwd_w<32, MC>(ck, ni, c->stream, it, pull, c->d_coarse, rhs, c->d_up, c->d_beff, sv);
      else
        launch_fwd_w<48, MC>(ck, ni, c->stream, it, pull, c->d_coarse, rhs, c->d_up, c->d_beff, sv);
    } else {
      hipLaunchKernelGGL(k_nd_fwd<MC>, dim3(ni), dim3(256), 0, c->stream, it, pull, c->d_coarse, rhs, c->d_up,
                         c->d_beff, sv);
    }
  }
  if (mid) hipEventRecord(mid, c->stream);
  // backward: the upper levels one launch each (LDS sized per level; the upper
  // levels' items were split when the lists were built), then the subtrees.
  // (A fused backward kernel over the same subtrees needs 137 KB of LDS at
  // 128^2: one workgroup per CU, two rounds of workgroups, slower than the
  // three-level subtree kernel.)
  const int btop = co.sub_level < L ? co.sub_level : L;
  for (int l = 0; l < btop; ++l) {
    const int i0 = co.bw_off[l], ni = co.bw_off[l + 1] - i0;
    if (ni == 0) continue;
    const NDItem* it = c->d_bw_items + i0;
    const int nf = std::max(1, co.lvl_nfmax[l]);
    const int nch = (nf + 63) / 64;
    if (co.lvl_bw_rows[l] == 16 && ni >= ND_WAVE_ITEMS && nch <= 4) {
      const dim3 grid((ni + 3) / 4);  // every load case in each workgroup
      if (nch <= 2)
        hipLaunchKernelGGL((k_nd_bwd_w<2, MC>), grid, dim3(256), 0, c->stream, it, ni, c->d_nd_bnd, c->d_coarse,
                           c->d_beff, x, sv);
      else if (nch <= 3)
        hipLaunchKernelGGL((k_nd_bwd_w<3, MC>), grid, dim3(256), 0, c->stream, it, ni, c->d_nd_bnd, c->d_coarse,
                           c->d_beff, x, sv);
      else
        hipLaunchKernelGGL((k_nd_bwd_w<4, MC>), grid, dim3(256), 0, c->stream, it, ni, c->d_nd_bnd, c->d_coarse,
                           c->d_beff, x, sv);
      continue;
    }
    const size_t lds = (size_t)((nf + 1023) / 1024 * 1024) * sizeof(double);
    if (co.lvl_bw_rows[l] == 4)
      launch_bwd<1, MC>(nch, ni, lds, c->stream, it, c->d_nd_bnd, c->d_coarse, c->d_beff, x, sv);
    else
      launch_bwd<ND_BW_ROWS / 4, MC>(nch, ni, lds, c->stream, it, c->d_nd_bnd, c->d_coarse, c->d_beff, x, sv);
  }
  if (co.sub_level < L) {
    const int nch = (std::max(1, co.sub_nfmax) + 63) / 64;
    const dim3 grid(co.sub_count);  // every load case in each workgroup
    if (nch <= 2)
      hipLaunchKernelGGL((k_nd_bwd_sub<2, MC>), grid, dim3(256), 0, c->stream, c->d_sub_bw_items, c->d_sub_bw_off,
                         co.sub_nst, c->d_nd_bnd, c->d_coarse, c->d_beff, x, sv);
    else if (nch <= 3)
      hipLaunchKernelGGL((k_nd_bwd_sub<3, MC>), grid, dim3(256), 0, c->stream, c->d_sub_bw_items, c->d_sub_bw_off,
                         co.sub_nst, c->d_nd_bnd, c->d_coarse, c->d_beff, x, sv);
    else
      hipLaunchKernelGGL((k_nd_bwd_sub<4, MC>), grid, dim3(256), 0, c->stream, c->d_sub_bw_items, c->d_sub_bw_off,
                         co.sub_nst, c->d_nd_bnd, c->d_coarse, c->d_beff, x, sv);
  }
  return hipGetLastError();
}

hipError_t launch_coarse_solve(Ctx* c, const double* rhs, double* x, hipEvent_t mid, int nr, unsigned mask) {
  const CoarseLayout& co = c->co;
  // the load cases' sweep vectors are laid out one after another with the
  // strides the context allocated
  const SweepVecs sv{(long long)c->NC, (long long)co.nd_up_total + 1, (long long)co.nd_beff_total + 1, mask, nr};
  return nr > 1 ? coarse_sweeps<true>(c, rhs, x, mid, sv) : coarse_sweeps<false>(c, rhs, x, mid, sv);
}

}  // namespace lbddc
