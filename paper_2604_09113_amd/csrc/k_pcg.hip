// Interface PCG with the BDDC preconditioner (A9; Sec. 3.3, Alg. 1) and the
// interior recovery (A10; Sec. 3.2).
//
// Per iteration:
//   q = S p            per cell: gather p (R_U), packed 64x64 product, partial;
//                      then a gather-sum over the <= 4 cells sharing each dof
//   z = S_BDDC^-1 r    per cell: gather r, fine correction (D-scaled explicit
//                      fine operator), coarse restriction Psi^T D r; coarse
//                      gather-sum, coarse solve, prolongation D Psi g; gather-sum
// The recurrence, residuals and S-products are FP64.  In the mixed path the
// fine operator and the coarse basis are stored and applied in FP32.
// Every sum runs in a fixed order (owner lists sorted by cell, block
// reductions with a fixed tree), so results are bitwise reproducible.
#include <chrono>

#include "internal.h"

namespace lbddc {

constexpr int kBlk = 256;

// The per-cell kernels below run one cell per 64-lane workgroup (NU <= 64):
// every lane first issues all of its loads of the cell's packed matrices (one
// coalesced sweep over the cell's block), then the block is staged in LDS and
// lane i forms row i.  A packed symmetric row is read as S[max(i,j)][min(i,j)]
// with a select in a single unrolled loop, so no lane diverges.

template <typename T, int N>
__device__ inline T sym_row(const T* __restrict__ Sp, const T* __restrict__ xs, int i) {
  const int ri = i * (i + 1) / 2;
  T s = 0;
#pragma unroll
  for (int j = 0; j < N; ++j) s += Sp[j <= i ? ri + j : j * (j + 1) / 2 + i] * xs[j];
  return s;
}

// Rows of a packed symmetric block times NR vectors in one pass over the row:
// s[k] = sum_j A[i][j] v[k][j], each sum in the order of sym_row (so every
// load case gets the same value as a product of its own)
template <typename T, int N, int NR, int LD>
__device__ inline void sym_rows(const T* __restrict__ Sp, const T (*v)[LD], int i, T (&s)[NR]) {
  const int ri = i * (i + 1) / 2;
#pragma unroll
  for (int k = 0; k < NR; ++k) s[k] = 0;
  // (several cases: a partial unroll, so that the vectors' LDS reads are not
  // all hoisted into registers)
  constexpr int U = NR == 1 ? N : 4;
#pragma unroll U
  for (int j = 0; j < N; ++j) {
    const T a = Sp[j <= i ? ri + j : j * (j + 1) / 2 + i];
#pragma unroll
    for (int k = 0; k < NR; ++k) s[k] += a * v[k][j];
  }
}

// y_i = S_i x_i for every cell and the load cases k < NR whose bit in mask is
// set (case k: vector x + k vs, partials part + k ps); S packed lower
// [nU(nU+1)/2], read once for all cases.  Only the cases in mask exist in
// memory: the others read case 0 and store nothing.
template <int NU, int NR>
__global__ __launch_bounds__(64) void k_op_local(const double* __restrict__ S, const int* __restrict__ RU,
                                                 const double* __restrict__ x, double* __restrict__ part,
                                                 long long vs, long long ps, unsigned mask) {
  static_assert(NU <= 64, "one row per lane");
  constexpr int NSP = NU * (NU + 1) / 2, NL = (NSP + 63) / 64;
  __shared__ double Ss[NL * 64];
  __shared__ double xs[NR][64];
  const int cell = blockIdx.x, l = threadIdx.x;
  const double* Sc = S + (size_t)cell * NSP;
  double v[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int i = l + 64 * k;
    v[k] = (i < NSP) ? Sc[i] : 0.0;
  }
  const int g = l < NU ? RU[(size_t)cell * NU + l] : -1;
  double xv[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) xv[k] = x[(((mask >> k) & 1u) ? k : 0) * vs + (g >= 0 ? g : 0)];  // inactive: case 0
#pragma unroll
  for (int k = 0; k < NR; ++k) xs[k][l] = g >= 0 ? xv[k] : 0.0;
#pragma unroll
  for (int k = 0; k < NL; ++k) Ss[l + 64 * k] = v[k];
  __syncthreads();
  if (l < NU) {
    double y[NR];
    sym_rows<double, NU, NR, 64>(Ss, xs, l, y);
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if ((mask >> k) & 1u) part[k * ps + (size_t)cell * NU + l] = y[k];
  }
}

// Sum over the 64 lanes of each of the 32 values v[0..31] a lane holds: a
// butterfly that halves the set of values a lane carries at every step (the
// lane with bit o set keeps the upper half and sends the lower, its partner
// the reverse), so 31 + 1 exchanges replace 32 separate reductions.  Value j
// ends in lanes 2j and 2j + 1 (the lane's bits 5..1 pick the halves).  The
// values live in a vector type, so that the per-lane choice of half stays a
// register select (an array here would be indexed through memory).
template <typename T>
using vec32 = T __attribute__((ext_vector_type(32)));
template <typename T>
__device__ __forceinline__ T wave_sum32(vec32<T> v) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int o = 32, m = 32; o >= 2; o >>= 1, m >>= 1) {
    const bool up = l & o;
#pragma unroll
    for (int k = 0; k < m / 2; ++k) {
      const T lo = v[k], hi = v[m / 2 + k];
      v[k] = (up ? hi : lo) + __shfl_xor(up ? lo : hi, o);
    }
  }
  return v[0] + __shfl_xor(v[0], 1);
}

// fine correction and coarse restriction of one cell (T = double or float):
// partU = [0; P r_E] (P packed over the nE = nU - 8 non-corner slots),
// partC = Psi^T r  (Psi stored column by column, [nC][nU]): lane i multiplies
// row i of Psi by r_i and the column sums are formed by wave_sum32.  P and Psi
// are read once for the load cases k < NR with their bit in mask set (case k:
// r + k vs, partU + k pu, partC + k pc).
template <typename T, int NU, int NC, int NR>
__global__ __launch_bounds__(64) void k_pre_local(const T* __restrict__ P, const T* __restrict__ Psi,
                                                  const int* __restrict__ RU, const double* __restrict__ r,
                                                  double* __restrict__ partU, double* __restrict__ partC,
                                                  long long vs, long long pu, long long pc, unsigned mask) {
  static_assert(NU <= 64 && NC <= 32, "lane mapping");
  constexpr int NE = NU - 8, NSP = NE * (NE + 1) / 2, NLP = (NSP + 63) / 64;
  __shared__ T Ps[NLP * 64];
  __shared__ T rs[NR][64];
  const int cell = blockIdx.x, l = threadIdx.x, lc = l < NU ? l : 0;
  const T* Pc = P + (size_t)cell * NSP;
  const T* Qc = Psi + (size_t)cell * NU * NC;
  T vp[NLP], vq[NC];
#pragma unroll
  for (int k = 0; k < NLP; ++k) {
    const int i = l + 64 * k;
    vp[k] = (i < NSP) ? Pc[i] : (T)0;
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) vq[j] = Qc[j * NU + lc];
  const int g = l < NU ? RU[(size_t)cell * NU + l] : -1;
  T rl[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const double rv = r[(((mask >> k) & 1u) ? k : 0) * vs + (g >= 0 ? g : 0)];  // inactive: case 0
    rl[k] = g >= 0 ? (T)rv : (T)0;
    rs[k][l] = rl[k];
  }
#pragma unroll
  for (int k = 0; k < NLP; ++k) Ps[l + 64 * k] = vp[k];
  __syncthreads();
  if (l < NU) {
    T y[NR];
    sym_rows<T, NE, NR, 64>(Ps, reinterpret_cast<const T(*)[64]>(&rs[0][8]), l >= 8 ? l - 8 : 0, y);
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if ((mask >> k) & 1u) partU[k * pu + (size_t)cell * NU + l] = l >= 8 ? (double)y[k] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (!((mask >> k) & 1u)) continue;
    vec32<T> v;
#pragma unroll
    for (int j = 0; j < 32; ++j) v[j] = j < NC ? vq[j] * rl[k] : (T)0;
    const T cj = wave_sum32<T>(v);
    if ((l & 1) == 0 && (l >> 1) < NC) partC[k * pc + (size_t)cell * NC + (l >> 1)] = (double)cj;
  }
}

// partU += Psi g_loc (coarse prolongation, D already folded into Psi); lane i
// forms row i, reading entry i of every column of the cell's Psi block once
// for the load cases k < NR with their bit in mask set (case k: g + k gs,
// partU + k pu)
template <typename T, int NU, int NC, int NR>
__global__ __launch_bounds__(64) void k_prolong(const T* __restrict__ Psi, const int* __restrict__ RC,
                                                const double* __restrict__ g, double* __restrict__ partU,
                                                long long gsd, long long pu, unsigned mask) {
  __shared__ T gs[NR][64];
  const int cell = blockIdx.x, l = threadIdx.x;
  T row[NC];
  if (l < NU) {
    const T* Qc = Psi + (size_t)cell * NU * NC + l;
#pragma unroll
    for (int j = 0; j < NC; ++j) row[j] = Qc[j * NU];
  }
  if (l < NC) {
    const int gc = RC[(size_t)cell * NC + l];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const double gv = g[(((mask >> k) & 1u) ? k : 0) * gsd + (gc >= 0 ? gc : 0)];  // inactive: case 0
      gs[k][l] = gc >= 0 ? (T)gv : (T)0;
    }
  }
  __syncthreads();
  if (l < NU) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (!((mask >> k) & 1u)) continue;
      T s = 0;
#pragma unroll
      for (int j = 0; j < NC; ++j) s += row[j] * gs[k][j];
      partU[k * pu + (size_t)cell * NU + l] += (double)s;
    }
  }
}

// block-level fixed-order sum of v (blockDim = kBlk = four waves): a
// butterfly of xor-shuffles within each wave, then the four wave sums in
// order; the result is valid in every thread
static_assert(kBlk == 256, "four waves per block");
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// out[g] = sum of owners' partials; optional partial dot out . w per block.
// Load cases k < nr with their bit in mask: part + k ps, out and w + k vs,
// red + k rs; the owner list is read once for all of them.
__global__ __launch_bounds__(kBlk) void k_gather_dot(const double* __restrict__ part, const int4* __restrict__ own4,
                                                     double* __restrict__ out, int N, const double* __restrict__ w,
                                                     double* __restrict__ red, long long ps = 0, long long vs = 0,
                                                     long long rs = 0, int nr = 1, unsigned mask = 1u) {
  __shared__ double sh[kBlk];
  const int g = blockIdx.x * kBlk + threadIdx.x, gc = g < N ? g : 0;
  // the owners in increasing cell order (a missing owner reads entry 0 and
  // adds nothing)
  const int4 o = own4[gc];
  const int i0 = o.x >= 0 ? o.x : 0, i1 = o.y >= 0 ? o.y : 0, i2 = o.z >= 0 ? o.z : 0, i3 = o.w >= 0 ? o.w : 0;
  for (int k = 0; k < nr; ++k) {
    if (!((mask >> k) & 1u)) continue;
    const double* pk = part + k * ps;
    // all four values requested at once, with w when a dot is asked for
    const double v0 = pk[i0], v1 = pk[i1], v2 = pk[i2], v3 = pk[i3];
    const double wv = red ? w[k * vs + gc] : 0.0;
    double s = 0.0;
    if (g < N) {
      if (o.x >= 0) s += v0;
      if (o.y >= 0) s += v1;
      if (o.z >= 0) s += v2;
      if (o.w >= 0) s += v3;
      out[k * vs + g] = s;
    }
    if (red) {
      double d = (g < N) ? s * wv : 0.0;
      d = block_sum(d, sh);
      if (threadIdx.x == 0) red[k * rs + blockIdx.x] = d;
      __syncthreads();  // sh is reused by the next case
    }
  }
}

// scal[dst] = sum of red[0..n) (fixed order, one block); then an optional ratio
// mode 0: plain sum; 1: alpha = scal[0] / sum (pq), flag if sum <= 0
// mode 2: rz_new = sum, beta = rz_new / scal[0], scal[0] = rz_new
__global__ __launch_bounds__(kBlk) void k_reduce(const double* __restrict__ red, int n, double* __restrict__ scal,
                                                 int dst, int mode) {
  __shared__ double sh[kBlk];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlk) s += red[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    scal[dst] = s;
    if (mode == 1) {
      if (!(s > 0.0)) scal[7] = 1.0;
      scal[2] = scal[0] / s;
    } else if (mode == 2) {
      if (!(s > 0.0)) scal[7] = 1.0;
      scal[5] = s / scal[0];
      scal[0] = s;
    }
  }
}

// The block path's step lengths, reduced once per load case (y = blockIdx.y,
// skipped unless its bit in mask is set) in the order of wg_sum, so every case
// gets the value its single-case solve computes inside the update kernels:
//   mode 1: pq = sum red (p.q partials), alpha = scal[rz_slot] / pq -> scal[1], scal[2]
//   mode 2: rz = sum red (r.z partials) -> scal[new_slot], beta = rz / scal[old_slot] -> scal[5]
//           (beta = 0 when init)
// A non-positive pq or rz sets scal[7].
__global__ __launch_bounds__(kBlk) void k_step_scalars(const double* __restrict__ red, int n, long long rs,
                                                       double* __restrict__ scal, long long ss, int mode, int slot_a,
                                                       int slot_b, int init, unsigned mask) {
  __shared__ double sh[kBlk];
  if (!((mask >> blockIdx.y) & 1u)) return;
  red += blockIdx.y * rs;
  scal += blockIdx.y * ss;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlk) s += red[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    if (mode == 1) {
      scal[1] = s;
      scal[2] = scal[slot_a] / s;
    } else {
      scal[slot_b] = s;
      scal[5] = init ? 0.0 : s / scal[slot_a];
    }
    if (!(s > 0.0)) scal[7] = 1.0;
  }
}

// ---- interface-vector kernels of the iteration: kVec entries per thread ----
constexpr int kVec = 4;
constexpr int kVB = kBlk * kVec;  // entries per workgroup

// fixed-order sum of red[0, n) by one workgroup; every workgroup that calls it
// on the same data gets the same value
__device__ inline double wg_sum(const double* __restrict__ red, int n, double* sh) {
  // each thread adds red[t], red[t + kBlk], ... in that order; the loads of
  // eight terms are issued together (clamped index, unused values discarded)
  double s = 0.0;
  for (int base = 0; base < n; base += 8 * kBlk) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = base + threadIdx.x + k * kBlk;
      v[k] = red[i < n ? i : 0];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (base + threadIdx.x + k * kBlk < n) s += v[k];
  }
  s = block_sum(s, sh);
  __syncthreads();
  return s;
}

// alpha = rz / (p.q) from the p.q partials (each workgroup sums them in the same
// order); x += alpha p; r -= alpha q; partial r.r per workgroup.  Workgroup 0
// records p.q and alpha and flags p.q <= 0 in scal[7].
// host: the pinned host buffer, as a device address: [7] breakdown flag,
// [32 + block] r.r partials (the host reads each slot once it has been written)
// Load case y = blockIdx.y (skipped unless its bit in mask is set): vectors
// + y vs, scalars + y ss, partials + y rs, host slots + y ss.
__global__ __launch_bounds__(kBlk) void k_update_xr4(double* __restrict__ x, double* __restrict__ r,
                                                     const double* __restrict__ p, const double* __restrict__ q,
                                                     double* __restrict__ scal, int N,
                                                     const double* __restrict__ red_pq, int nred, int rz_slot,
                                                     double* __restrict__ host, long long vs = 0, long long ss = 0,
                                                     long long rs = 0, unsigned mask = 1u) {
  __shared__ double sh[kBlk];
  if (!((mask >> blockIdx.y) & 1u)) return;
  x += blockIdx.y * vs;
  r += blockIdx.y * vs;
  p += blockIdx.y * vs;
  q += blockIdx.y * vs;
  scal += blockIdx.y * ss;
  red_pq += blockIdx.y * rs;
  host += blockIdx.y * ss;
  // the vector entries are requested first (clamped index) and arrive while
  // the workgroup sums the p.q partials
  const int g0 = blockIdx.x * kVB + threadIdx.x;
  double xv[kVec], pv[kVec], rv[kVec], qv[kVec];
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const int g = g0 + j * kBlk, gc = g < N ? g : 0;
    xv[j] = x[gc];
    pv[j] = p[gc];
    rv[j] = r[gc];
    qv[j] = q[gc];
  }
  // nred = 0: alpha already reduced (k_step_scalars)
  const double pq = nred ? wg_sum(red_pq, nred, sh) : scal[1];
  const double alpha = nred ? scal[rz_slot] / pq : scal[2];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (nred) {
      scal[1] = pq;
      scal[2] = alpha;
      if (!(pq > 0.0)) scal[7] = 1.0;
    }
    host[7] = scal[7];
  }
  double d = 0.0;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const int g = g0 + j * kBlk;
    if (g < N) {
      x[g] = xv[j] + alpha * pv[j];
      const double rn = rv[j] - alpha * qv[j];
      r[g] = rn;
      d += rn * rn;
    }
  }
  d = block_sum(d, sh);
  if (threadIdx.x == 0) host[32 + blockIdx.x] = d;
}

// rz_new from the r.z partials; p = z (init) or z + beta p with
// beta = rz_new / scal[old_slot]; workgroup 0 stores rz_new in scal[new_slot]
// (a different slot, so no workgroup reads a value being replaced) and flags
// rz_new <= 0 in scal[7].
// (load case y = blockIdx.y as in k_update_xr4)
__global__ __launch_bounds__(kBlk) void k_update_p4(double* __restrict__ p, const double* __restrict__ z,
                                                    double* __restrict__ scal, int N,
                                                    const double* __restrict__ red_rz, int nred, int old_slot,
                                                    int new_slot, int init, long long vs = 0, long long ss = 0,
                                                    long long rs = 0, unsigned mask = 1u) {
  __shared__ double sh[kBlk];
  if (!((mask >> blockIdx.y) & 1u)) return;
  p += blockIdx.y * vs;
  z += blockIdx.y * vs;
  scal += blockIdx.y * ss;
  red_rz += blockIdx.y * rs;
  // z and p requested first (clamped index), while the r.z partials are summed
  const int g0 = blockIdx.x * kVB + threadIdx.x;
  double zv[kVec], pv[kVec];
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const int g = g0 + j * kBlk, gc = g < N ? g : 0;
    zv[j] = z[gc];
    pv[j] = p[gc];
  }
  // nred = 0: rz and beta already reduced (k_step_scalars)
  const double rz = nred ? wg_sum(red_rz, nred, sh) : scal[new_slot];
  const double beta = nred ? (init ? 0.0 : rz / scal[old_slot]) : scal[5];
  if (nred && blockIdx.x == 0 && threadIdx.x == 0) {
    scal[new_slot] = rz;
    scal[5] = beta;
    if (!(rz > 0.0)) scal[7] = 1.0;
  }
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const int g = g0 + j * kBlk;
    if (g < N) p[g] = init ? zv[j] : zv[j] + beta * pv[j];
  }
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int N) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < N) dst[g] = src[g];
}

__global__ void k_dot(const double* __restrict__ a, const double* __restrict__ b, int N, double* __restrict__ red) {
  __shared__ double sh[kBlk];
  int g = blockIdx.x * kBlk + threadIdx.x;
  double d = g < N ? a[g] * b[g] : 0.0;
  d = block_sum(d, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = d;
}

// ---- interior recovery (tractions act on skeleton dofs only)
// The interior dofs of one cell per 64-lane wave from the multipliers W of
// the blocked elimination in the local Schur kernel: interior panels from the
// last to the first, u_p = -sum_{i > p} W_(p,i)^T u_i over the tiles below
// panel p (interior and skeleton dofs padded to 16-row tiles, the padding
// zero).  The padded cell vector lives in LDS.  Lane 16 g + c multiplies the
// W entries (row c, columns g + 4v) of each tile, read contiguously across
// the lanes, by u of row c; the 16 lanes of row g then sum their partials,
// and the panel's 16 values go to LDS for the panels above.
template <int P>
__global__ __launch_bounds__(64) void k_recover(const double* __restrict__ W, const int* __restrict__ RU,
                                                const double* __restrict__ x, int nx, int Gx,
                                                double* __restrict__ u, double* __restrict__ ucell) {
  constexpr int NI = 2 * (P - 1) * (P - 1), NU = 8 * P, NDOF = 2 * (P + 1) * (P + 1);
  constexpr int NIP = (NI + 15) / 16, NT = NIP + (NU + 15) / 16;
  const int cell = blockIdx.x, l = threadIdx.x, g = l >> 4, c = l & 15;
  __shared__ double ub[16 * NT];
  for (int i = l; i < 16 * NT; i += 64) {
    const int s = i - 16 * NIP;
    double v = 0.0;
    if (s >= 0 && s < NU) {
      const int gi = RU[(size_t)cell * NU + s];
      v = gi >= 0 ? x[gi] : 0.0;
    }
    ub[i] = v;
  }
  __syncthreads();
  const double* Wc = W + (size_t)cell * schur_w_count(P);
  for (int p = NIP - 1; p >= 0; --p) {
    const double* Wp = Wc + 256 * (p * (NT - 1) - p * (p - 1) / 2);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // tiles p + 1 .. NT - 1, all loads in flight (past the last tile: tile
    // p + 1 again, times zero)
#pragma unroll
    for (int t = 0; t < NT - 1; ++t) {
      const bool in = p + 1 + t < NT;
      const int tc = in ? t : 0;
      const double ut = in ? ub[16 * (p + 1 + t) + c] : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = fma(Wp[256 * tc + 64 * v + l], ut, acc[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) acc[v] += __shfl_xor(acc[v], o, 16);
    if (c == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) ub[16 * p + g + 4 * v] = -acc[v];
    }
    __syncthreads();
  }
  const int ix = cell % nx, iy = cell / nx;
  for (int k = l; k < NI; k += 64) {
    const double v = ub[k];
    const int n = k >> 1, comp = k & 1;
    const int a = n % (P - 1) + 1, b = n / (P - 1) + 1;
    u[((size_t)(P * iy + b) * Gx + P * ix + a) * 2 + comp] = v;
    if (ucell) ucell[(size_t)cell * NDOF + k] = v;
  }
  if (ucell)
    for (int s = l; s < NU; s += 64) ucell[(size_t)cell * NDOF + NI + s] = ub[16 * NIP + s];
}

__global__ void k_scatter_skel(const double* __restrict__ x, const int* __restrict__ node, int NU,
                               double* __restrict__ u) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= NU) return;
  u[(size_t)node[g >> 1] * 2 + (g & 1)] = x[g];
}

__global__ void k_fill_p(double* __restrict__ x, long long n, double v) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) x[i] = v;
}

// partial sums of (a - b)^2
__global__ void k_diff_dot(const double* __restrict__ a, const double* __restrict__ b, int N, double* __restrict__ red) {
  __shared__ double sh[kBlk];
  int g = blockIdx.x * kBlk + threadIdx.x;
  double d = g < N ? (a[g] - b[g]) : 0.0;
  d = block_sum(d * d, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = d;
}

// ---------------------------------------------------------------------------
// The per-cell kernels of a block of nr load cases (vectors NU apart, cell
// partials ncell nU (fine) and ncell nC (coarse) apart, coarse vectors NC
// apart): NR = 1 for a single case, 8 otherwise (the mask selects the cases).
template <int NU, int NC, int NR>
static void launch_pre(Ctx* c, bool fp32, const double* r, unsigned mask) {
  const long long vs = c->NU, pu = (long long)c->ncell * c->nU, pc = (long long)c->ncell * c->nC;
  if (fp32)
    hipLaunchKernelGGL((k_pre_local<float, NU, NC, NR>), dim3(c->ncell), dim3(64), 0, c->stream,
                       (const float*)c->d_P, (const float*)c->d_Psi, c->d_RU, r, c->d_partU, c->d_partC, vs, pu, pc,
                       mask);
  else
    hipLaunchKernelGGL((k_pre_local<double, NU, NC, NR>), dim3(c->ncell), dim3(64), 0, c->stream,
                       (const double*)c->d_P, (const double*)c->d_Psi, c->d_RU, r, c->d_partU, c->d_partC, vs, pu,
                       pc, mask);
}
template <int NU, int NC, int NR>
static void launch_prolong(Ctx* c, bool fp32, unsigned mask) {
  const long long gs = c->NC, pu = (long long)c->ncell * c->nU;
  if (fp32)
    hipLaunchKernelGGL((k_prolong<float, NU, NC, NR>), dim3(c->ncell), dim3(64), 0, c->stream,
                       (const float*)c->d_Psi, c->d_RC, c->d_xc, c->d_partU, gs, pu, mask);
  else
    hipLaunchKernelGGL((k_prolong<double, NU, NC, NR>), dim3(c->ncell), dim3(64), 0, c->stream,
                       (const double*)c->d_Psi, c->d_RC, c->d_xc, c->d_partU, gs, pu, mask);
}

#define DISPATCH_P(macro) \
  switch (c->p) { macro(2) macro(3) macro(4) macro(5) macro(6) macro(7) macro(8) default: break; }

static void op_local(Ctx* c, const double* x, bool blk = false, unsigned mask = 1u) {
  const long long vs = c->NU, ps = (long long)c->ncell * c->nU;
#define OPC(pp)                                                                                               \
  case pp:                                                                                                    \
    if (blk)                                                                                                  \
      hipLaunchKernelGGL((k_op_local<8 * pp, kBlockRhs>), dim3(c->ncell), dim3(64), 0, c->stream, c->d_S,     \
                         c->d_RU, x, c->d_partU, vs, ps, mask);                                               \
    else                                                                                                      \
      hipLaunchKernelGGL((k_op_local<8 * pp, 1>), dim3(c->ncell), dim3(64), 0, c->stream, c->d_S, c->d_RU, x, \
                         c->d_partU, vs, ps, 1u);                                                             \
    break;
  DISPATCH_P(OPC)
#undef OPC
}
static void pre_local(Ctx* c, bool fp32, const double* r, bool blk = false, unsigned mask = 1u) {
#define PRC(pp)                                                                 \
  case pp:                                                                      \
    if (blk) {                                                                  \
      if (c->nce == 3) launch_pre<8 * pp, 20, kBlockRhs>(c, fp32, r, mask);     \
      else launch_pre<8 * pp, 16, kBlockRhs>(c, fp32, r, mask);                 \
    } else {                                                                    \
      if (c->nce == 3) launch_pre<8 * pp, 20, 1>(c, fp32, r, 1u);               \
      else launch_pre<8 * pp, 16, 1>(c, fp32, r, 1u);                           \
    }                                                                           \
    break;
  DISPATCH_P(PRC)
#undef PRC
}
static void prolong(Ctx* c, bool fp32, bool blk = false, unsigned mask = 1u) {
#define PLC(pp)                                                                 \
  case pp:                                                                      \
    if (blk) {                                                                  \
      if (c->nce == 3) launch_prolong<8 * pp, 20, kBlockRhs>(c, fp32, mask);    \
      else launch_prolong<8 * pp, 16, kBlockRhs>(c, fp32, mask);                \
    } else {                                                                    \
      if (c->nce == 3) launch_prolong<8 * pp, 20, 1>(c, fp32, 1u);              \
      else launch_prolong<8 * pp, 16, 1>(c, fp32, 1u);                          \
    }                                                                           \
    break;
  DISPATCH_P(PLC)
#undef PLC
}

// With LBDDC_TIME_SAMPLE, one operator launch and one preconditioner
// application in kSample record events (kRing is a multiple of kSample).
constexpr int kSample = 8;
static_assert(Ctx::kRing % kSample == 0, "a ring slot is timed on every use or never");

// Device times of the timed PCG phases, accumulated from the event ring.
struct PhaseAcc {
  double op = 0, pre = 0, coarse = 0, cf = 0, cb = 0;
};

// The host learns that an iteration's update has finished from the pinned
// buffer it writes (coherent host memory, so the stores reach the host
// directly), not from an event: an event marker between two kernels leaves
// the device idle for several microseconds.  Before the update is enqueued
// the host fills its slots (breakdown flag 7, r.r partials 32 ..) with a
// signalling-NaN pattern; arithmetic produces only quiet NaNs, so a slot that
// no longer holds the pattern has been written.
constexpr unsigned long long kUnset = 0x7ff4c0ffee5e7f11ull;
static inline int hred_slot(int k) { return k == 0 ? 7 : 31 + k; }  // k = 0 .. nv

static void hred_unset(Ctx* c, int nv) {
  for (int k = 0; k <= nv; ++k)
    __atomic_store_n(reinterpret_cast<unsigned long long*>(c->h_red + hred_slot(k)), kUnset, __ATOMIC_RELAXED);
}

// Spin until every slot is written.  The spin is bounded: past 50 ms the
// stream is synchronised instead (which also reports a device error); a slot
// still unset once everything enqueued has finished is an error.
static hipError_t hred_wait(Ctx* c, int nv) {
  auto written = [&](int k) {
    return __atomic_load_n(reinterpret_cast<const unsigned long long*>(c->h_red + hred_slot(k)), __ATOMIC_ACQUIRE) !=
           kUnset;
  };
  const auto t0 = std::chrono::steady_clock::now();
  int k = 0;
  for (unsigned spins = 0;; ++spins) {
    while (k <= nv && written(k)) ++k;
    if (k > nv) return hipSuccess;
    if ((spins & 1023u) == 1023u && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
      const hipError_t e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return e;
      while (k <= nv && written(k)) ++k;
      return k > nv ? hipSuccess : hipErrorLaunchFailure;
    }
  }
}

static double elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms : 0.0;
}

// read back ring slot `s` of an operator launch / a preconditioner application
static void harvest_op(Ctx* c, int s, PhaseAcc& a) {
  if (!(c->timing & LBDDC_TIME_OP)) return;
  hipEventSynchronize(c->pev[s][1]);
  a.op += elapsed(c->pev[s][0], c->pev[s][1]);
}
static void harvest_apply(Ctx* c, int s, PhaseAcc& a) {
  hipEvent_t* e = c->pev[s];
  if (c->timing & LBDDC_TIME_PRE) {
    hipEventSynchronize(e[3]);
    a.pre += elapsed(e[2], e[3]);
  }
  if (c->timing & LBDDC_TIME_COARSE) {
    hipEventSynchronize(e[6]);
    a.coarse += elapsed(e[4], e[6]);
    a.cf += elapsed(e[4], e[5]);
    a.cb += elapsed(e[5], e[6]);
  }
}

// z = S_BDDC^-1 r (Alg. 1), with the partial dot r.z into red; the timed
// phases record their events into ring slot `slot`
// (block: the nr load cases of the context's block buffers with their bit in
// mask set, z and r NU apart, red vred_stride apart)
static hipError_t apply_M(Ctx* c, bool fp32, const double* r, double* z, double* red, int slot, bool timed,
                          int nr = 1, unsigned mask = 1u) {
  const int nbU = (c->NU + kBlk - 1) / kBlk, nbC = (c->NC + kBlk - 1) / kBlk;
  const bool blk = nr > 1;
  const long long pu = (long long)c->ncell * c->nU, pc = (long long)c->ncell * c->nC;
  hipEvent_t* e = c->pev[slot];
  const bool tp = timed && (c->timing & LBDDC_TIME_PRE), tc = timed && (c->timing & LBDDC_TIME_COARSE);
  if (tp) hipEventRecord(e[2], c->stream);
  pre_local(c, fp32, r, blk, mask);
  if (tp) hipEventRecord(e[3], c->stream);
  hipLaunchKernelGGL(k_gather_dot, dim3(nbC), dim3(kBlk), 0, c->stream, c->d_partC, c->d_cown4, c->d_zc, c->NC,
                     (const double*)nullptr, (double*)nullptr, pc, (long long)c->NC, 0LL, nr, mask);
  if (tc) hipEventRecord(e[4], c->stream);
  hipError_t err = launch_coarse_solve(c, c->d_zc, c->d_xc, tc ? e[5] : nullptr, nr, mask);
  if (err != hipSuccess) return err;
  if (tc) hipEventRecord(e[6], c->stream);
  prolong(c, fp32, blk, mask);
  hipLaunchKernelGGL(k_gather_dot, dim3(nbU), dim3(kBlk), 0, c->stream, c->d_partU, c->d_uown4, z, c->NU, r, red,
                     pu, (long long)c->NU, (long long)c->vred_stride(), nr, mask);
  return hipGetLastError();
}

hipError_t pcg_solve(Ctx* c, int rhs, double rtol, int max_iter, lbddc_solve_info* info, bool fp32, double* t_op,
                     double* t_pre, double* t_coarse, double* t_cfwd, double* t_cbwd, int* n_apply) {
  const int N = c->NU, nb = (N + kBlk - 1) / kBlk, nv = (N + kVB - 1) / kVB;
  double* f = c->d_f + (size_t)rhs * N;
  double* x = c->d_x + (size_t)rhs * N;
  double *r = c->d_r, *z = c->d_z, *p = c->d_p, *q = c->d_q;
  double* red = c->d_red;
  // partials: p.q and r.z per gather workgroup (nb); r.r per update workgroup
  // (nv) right after the scalar slots, so that one copy brings both to the host
  double *red_pq = c->d_vred, *red_rz = c->d_vred + nb;
  double* scal = c->d_scal;
  // scalar slots: 1 p.q, 2 alpha, 5 beta, 6 f.f, 7 breakdown flag, 10/11 r.z (alternating)
  hipLaunchKernelGGL(k_fill_p, dim3(256), dim3(256), 0, c->stream, x, (long long)N, 0.0);
  hipLaunchKernelGGL(k_fill_p, dim3(1), dim3(64), 0, c->stream, scal, 16LL, 0.0);
  hipLaunchKernelGGL(k_copy, dim3(nb), dim3(kBlk), 0, c->stream, r, f, N);
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBlk), 0, c->stream, f, f, N, red);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlk), 0, c->stream, red, nb, scal, 6, 0);
  // event ring: an operator launch and a preconditioner application use slot
  // (count mod kRing); a slot is read back before it is recorded again, by
  // which time its events completed long ago, and the rest after the loop
  PhaseAcc acc;
  int napp = 0, nop = 0;
  // with LBDDC_TIME_SAMPLE only operator launches and applications whose count
  // is a multiple of kSample record events, and the totals are scaled to all
  const int every = (c->timing & LBDDC_TIME_SAMPLE) ? kSample : 1;
  auto timed = [&](int k) { return k % every == 0; };
  auto apply = [&](void) -> hipError_t {
    const int sl = napp % Ctx::kRing;
    if (napp >= Ctx::kRing && timed(napp - Ctx::kRing)) harvest_apply(c, sl, acc);
    const bool tm = timed(napp);
    ++napp;
    return apply_M(c, fp32, r, z, red_rz, sl, tm);
  };
  auto finish = [&](hipError_t e) {
    for (int k = std::max(0, napp - Ctx::kRing); k < napp; ++k)
      if (timed(k)) harvest_apply(c, k % Ctx::kRing, acc);
    for (int k = std::max(0, nop - Ctx::kRing); k < nop; ++k)
      if (timed(k)) harvest_op(c, k % Ctx::kRing, acc);
    const int napp_t = (napp + every - 1) / every, nop_t = (nop + every - 1) / every;
    const double sa = napp_t ? (double)napp / napp_t : 0.0, so = nop_t ? (double)nop / nop_t : 0.0;
    if (t_op) *t_op += acc.op * so;
    if (t_pre) *t_pre += acc.pre * sa;
    if (t_coarse) *t_coarse += acc.coarse * sa;
    if (t_cfwd) *t_cfwd += acc.cf * sa;
    if (t_cbwd) *t_cbwd += acc.cb * sa;
    if (n_apply) *n_apply += napp;
    return e;
  };
  int slot = 10;
  hipError_t e = apply();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_update_p4, dim3(nv), dim3(kBlk), 0, c->stream, p, z, scal, N, red_rz, nb, slot, slot, 1);
  e = hipMemcpyAsync(c->h_scal, scal, 16 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  const double ff = c->h_scal[6];
  double rel = 1.0;
  int it = 0;
  info->iters = 0;
  info->rel_res = ff > 0 ? 1.0 : 0.0;
  if (!(ff > 0)) return finish(hipSuccess);
  if (c->h_scal[7] != 0.0) return finish(hipErrorUnknown);  // breakdown, reported by the caller
  const bool top = c->timing & LBDDC_TIME_OP;
  while (it < max_iter) {
    hred_unset(c, nv);
    const int so = nop % Ctx::kRing;
    if (nop >= Ctx::kRing && timed(nop - Ctx::kRing)) harvest_op(c, so, acc);
    const bool tm = top && timed(nop);
    ++nop;
    if (tm) hipEventRecord(c->pev[so][0], c->stream);
    op_local(c, p);
    if (tm) hipEventRecord(c->pev[so][1], c->stream);
    hipLaunchKernelGGL(k_gather_dot, dim3(nb), dim3(kBlk), 0, c->stream, c->d_partU, c->d_uown4, q, N,
                       p, red_pq);
    hipLaunchKernelGGL(k_update_xr4, dim3(nv), dim3(kBlk), 0, c->stream, x, r, p, q, scal, N, red_pq, nb, slot,
                       c->d_hred);
    // speculatively enqueue the preconditioner and the direction update of the next iteration
    e = apply();
    if (e != hipSuccess) return e;
    const int next = slot == 10 ? 11 : 10;
    hipLaunchKernelGGL(k_update_p4, dim3(nv), dim3(kBlk), 0, c->stream, p, z, scal, N, red_rz, nb, slot, next, 0);
    slot = next;
    e = hred_wait(c, nv);
    if (e != hipSuccess) return e;
    ++it;
    if (c->h_red[7] != 0.0) {
      hipStreamSynchronize(c->stream);
      info->iters = it;
      info->rel_res = rel;
      return finish(hipErrorUnknown);  // breakdown, reported by the caller
    }
    double rr = 0.0;  // r.r: the workgroup partials summed on the host in fixed order
    for (int i = 0; i < nv; ++i) rr += c->h_red[32 + i];
    rel = sqrt(rr / ff);
    if (rel <= rtol) break;
  }
  e = hipStreamSynchronize(c->stream);
  info->iters = it;
  info->rel_res = rel;
  return finish(e);
}

// PCG on the load cases r0 .. r0 + nr - 1 (nr <= kBlockRhs) as one block:
// every iteration makes one pass over S_i, the preconditioner's cell data and
// the coarse factor for all cases that have not converged.  Each case runs
// its own recurrence with its own scalars (the case's slice of the block
// buffers), in the same kernels and summation orders as a single-case solve,
// so its iterates and iteration count are those of pcg_solve.  A case stops
// (its bit leaves the mask, so no kernel touches its x again) at the first
// iteration whose residual meets rtol.  On a breakdown of any case the solve
// stops and returns hipErrorUnknown with the infos filled so far.
hipError_t pcg_solve_block(Ctx* c, int r0, int nr, double rtol, int max_iter, lbddc_solve_info* info, bool fp32,
                           double* t_op, double* t_pre, double* t_coarse, double* t_cfwd, double* t_cbwd,
                           int* n_apply, int* n_op) {
  const int N = c->NU, nb = (N + kBlk - 1) / kBlk, nv = (N + kVB - 1) / kVB;
  const long long VS = N, SS = (long long)c->scal_stride(), RS = (long long)c->vred_stride();
  double* f = c->d_f + (size_t)r0 * N;
  double* x = c->d_x + (size_t)r0 * N;
  double *r = c->d_r, *z = c->d_z, *p = c->d_p, *q = c->d_q;
  double *red_pq = c->d_vred, *red_rz = c->d_vred + nb;
  double* scal = c->d_scal;
  for (int k = 0; k < nr; ++k) {
    hipLaunchKernelGGL(k_fill_p, dim3(256), dim3(256), 0, c->stream, x + k * VS, (long long)N, 0.0);
    hipLaunchKernelGGL(k_fill_p, dim3(1), dim3(64), 0, c->stream, scal + k * SS, 16LL, 0.0);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(kBlk), 0, c->stream, r + k * VS, f + k * VS, N);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBlk), 0, c->stream, f + k * VS, f + k * VS, N, c->d_red);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlk), 0, c->stream, c->d_red, nb, scal + k * SS, 6, 0);
  }
  unsigned mask = (1u << nr) - 1u;
  PhaseAcc acc;
  int napp = 0, nop = 0;
  const int every = (c->timing & LBDDC_TIME_SAMPLE) ? kSample : 1;
  auto timed = [&](int k) { return k % every == 0; };
  auto apply = [&](void) -> hipError_t {
    const int sl = napp % Ctx::kRing;
    if (napp >= Ctx::kRing && timed(napp - Ctx::kRing)) harvest_apply(c, sl, acc);
    const bool tm = timed(napp);
    ++napp;
    return apply_M(c, fp32, r, z, red_rz, sl, tm, nr, mask);
  };
  auto finish = [&](hipError_t e) {
    for (int k = std::max(0, napp - Ctx::kRing); k < napp; ++k)
      if (timed(k)) harvest_apply(c, k % Ctx::kRing, acc);
    for (int k = std::max(0, nop - Ctx::kRing); k < nop; ++k)
      if (timed(k)) harvest_op(c, k % Ctx::kRing, acc);
    const int napp_t = (napp + every - 1) / every, nop_t = (nop + every - 1) / every;
    const double sa = napp_t ? (double)napp / napp_t : 0.0, so = nop_t ? (double)nop / nop_t : 0.0;
    if (t_op) *t_op += acc.op * so;
    if (t_pre) *t_pre += acc.pre * sa;
    if (t_coarse) *t_coarse += acc.coarse * sa;
    if (t_cfwd) *t_cfwd += acc.cf * sa;
    if (t_cbwd) *t_cbwd += acc.cb * sa;
    if (n_apply) *n_apply += napp;
    if (n_op) *n_op += nop;
    return e;
  };
  int slot = 10;
  hipError_t e = apply();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_step_scalars, dim3(1, nr), dim3(kBlk), 0, c->stream, red_rz, nb, RS, scal, SS, 2, slot, slot,
                     1, mask);
  hipLaunchKernelGGL(k_update_p4, dim3(nv, nr), dim3(kBlk), 0, c->stream, p, z, scal, N, red_rz, 0, slot, slot, 1,
                     VS, SS, RS, mask);
  std::vector<double> hs((size_t)nr * SS);
  e = hipMemcpyAsync(hs.data(), scal, hs.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  std::vector<double> ff(nr), rel(nr, 1.0);
  bool broke = false;
  for (int k = 0; k < nr; ++k) {
    ff[k] = hs[k * SS + 6];
    info[k] = lbddc_solve_info{0, ff[k] > 0 ? 1.0 : 0.0, 0};
    if (!(ff[k] > 0)) mask &= ~(1u << k);
    else if (hs[k * SS + 7] != 0.0) broke = true;
  }
  if (broke) return finish(hipErrorUnknown);
  // the pinned poll slots of case k: its breakdown flag and r.r partials
  double* hk = c->h_red;
  auto unset = [&](unsigned m) {
    for (int k = 0; k < nr; ++k)
      if ((m >> k) & 1u)
        for (int i = 0; i <= nv; ++i)
          __atomic_store_n(reinterpret_cast<unsigned long long*>(hk + k * SS + hred_slot(i)), kUnset, __ATOMIC_RELAXED);
  };
  auto wait = [&](unsigned m) -> hipError_t {
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spins = 0;; ++spins) {
      bool all = true;
      for (int k = 0; k < nr && all; ++k)
        if ((m >> k) & 1u)
          for (int i = 0; i <= nv && all; ++i)
            all = __atomic_load_n(reinterpret_cast<const unsigned long long*>(hk + k * SS + hred_slot(i)),
                                  __ATOMIC_ACQUIRE) != kUnset;
      if (all) return hipSuccess;
      if ((spins & 1023u) == 1023u && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
        const hipError_t er = hipStreamSynchronize(c->stream);
        if (er != hipSuccess) return er;
        for (int k = 0; k < nr; ++k)
          if ((m >> k) & 1u)
            for (int i = 0; i <= nv; ++i)
              if (__atomic_load_n(reinterpret_cast<const unsigned long long*>(hk + k * SS + hred_slot(i)),
                                  __ATOMIC_ACQUIRE) == kUnset)
                return hipErrorLaunchFailure;
        return hipSuccess;
      }
    }
  };
  const bool top = c->timing & LBDDC_TIME_OP;
  int it = 0;
  while (mask && it < max_iter) {
    unset(mask);
    const int so = nop % Ctx::kRing;
    if (nop >= Ctx::kRing && timed(nop - Ctx::kRing)) harvest_op(c, so, acc);
    const bool tm = top && timed(nop);
    ++nop;
    if (tm) hipEventRecord(c->pev[so][0], c->stream);
    op_local(c, p, true, mask);
    if (tm) hipEventRecord(c->pev[so][1], c->stream);
    hipLaunchKernelGGL(k_gather_dot, dim3(nb), dim3(kBlk), 0, c->stream, c->d_partU, c->d_uown4, q, N, p, red_pq,
                       (long long)c->ncell * c->nU, VS, RS, nr, mask);
    hipLaunchKernelGGL(k_step_scalars, dim3(1, nr), dim3(kBlk), 0, c->stream, red_pq, nb, RS, scal, SS, 1, slot, 0,
                       0, mask);
    hipLaunchKernelGGL(k_update_xr4, dim3(nv, nr), dim3(kBlk), 0, c->stream, x, r, p, q, scal, N, red_pq, 0, slot,
                       c->d_hred, VS, SS, RS, mask);
    // speculatively enqueue the preconditioner and the direction update of the next iteration
    e = apply();
    if (e != hipSuccess) return e;
    const int next = slot == 10 ? 11 : 10;
    hipLaunchKernelGGL(k_step_scalars, dim3(1, nr), dim3(kBlk), 0, c->stream, red_rz, nb, RS, scal, SS, 2, slot,
                       next, 0, mask);
    hipLaunchKernelGGL(k_update_p4, dim3(nv, nr), dim3(kBlk), 0, c->stream, p, z, scal, N, red_rz, 0, slot, next,
                       0, VS, SS, RS, mask);
    slot = next;
    e = wait(mask);
    if (e != hipSuccess) return e;
    ++it;
    for (int k = 0; k < nr; ++k) {
      if (!((mask >> k) & 1u)) continue;
      if (hk[k * SS + 7] != 0.0) broke = true;
      double rr = 0.0;  // r.r: the workgroup partials summed on the host in fixed order
      for (int i = 0; i < nv; ++i) rr += hk[k * SS + 32 + i];
      rel[k] = sqrt(rr / ff[k]);
      info[k].iters = it;
      info[k].rel_res = rel[k];
      if (rel[k] <= rtol) mask &= ~(1u << k);
    }
    if (broke) {
      hipStreamSynchronize(c->stream);
      return finish(hipErrorUnknown);  // breakdown, reported by the caller
    }
  }
  e = hipStreamSynchronize(c->stream);
  return finish(e);
}

// ||f - S x||_2 / ||f||_2 recomputed from the iterate
hipError_t pcg_true_residual(Ctx* c, int rhs, double* out) {
  const int N = c->NU, nb = (N + kBlk - 1) / kBlk;
  const double* f = c->d_f + (size_t)rhs * N;
  const double* x = c->d_x + (size_t)rhs * N;
  op_local(c, x);
  hipLaunchKernelGGL(k_gather_dot, dim3(nb), dim3(kBlk), 0, c->stream, c->d_partU, c->d_uown4, c->d_q,
                     N, (const double*)nullptr, (double*)nullptr);
  hipLaunchKernelGGL(k_diff_dot, dim3(nb), dim3(kBlk), 0, c->stream, f, c->d_q, N, c->d_red);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlk), 0, c->stream, c->d_red, nb, c->d_scal, 8, 0);
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBlk), 0, c->stream, f, f, N, c->d_red);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlk), 0, c->stream, c->d_red, nb, c->d_scal, 9, 0);
  hipError_t e = hipMemcpyAsync(c->h_scal, c->d_scal, 16 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  *out = c->h_scal[9] > 0 ? sqrt(c->h_scal[8] / c->h_scal[9]) : 0.0;
  return e;
}

// f_r = sum over owners of the cell loads (tractions act on skeleton dofs only)
hipError_t gather_rhs(Ctx* c, int rhs) {
  const int N = c->NU;
  hipLaunchKernelGGL(k_gather_dot, dim3((N + kBlk - 1) / kBlk), dim3(kBlk), 0, c->stream,
                     c->d_load + (size_t)rhs * c->ncell * c->nU, c->d_uown4, c->d_f + (size_t)rhs * N,
                     N, (const double*)nullptr, (double*)nullptr);
  return hipGetLastError();
}

hipError_t launch_recover(Ctx* c, int rhs) {
  const size_t nu = (size_t)c->Gx * c->Gy * 2;
  double* u = c->d_u + (size_t)rhs * nu;
  hipLaunchKernelGGL(k_fill_p, dim3(512), dim3(256), 0, c->stream, u, (long long)nu, 0.0);
  const double* x = c->d_x + (size_t)rhs * c->NU;
  double* uc = c->d_ucell ? c->d_ucell + (size_t)rhs * c->ncell * c->ndof : nullptr;
#define RCC(pp) case pp: hipLaunchKernelGGL(k_recover<pp>, dim3(c->ncell), dim3(64), 0, c->stream, c->d_W, c->d_RU, x, c->nx, c->Gx, u, uc); break;
  DISPATCH_P(RCC)
#undef RCC
  hipLaunchKernelGGL(k_scatter_skel, dim3((c->NU + 255) / 256), dim3(256), 0, c->stream, x, c->d_skel_node, c->NU, u);
  return hipGetLastError();
}

}  // namespace lbddc
