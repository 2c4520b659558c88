// Local Schur complement (A4, Sec. 3.2): S = K_UU - K_UI K_II^-1 K_IU, by
// blocked elimination of the interior dofs, sixteen at a time.
//
// The cell matrix in the dof order [interior | skeleton], each part padded
// with decoupled identity rows to a multiple of 16 (NIP interior and NUT
// skeleton tile rows, NT = NIP + NUT), is held as 16 x 16 tiles.  Interior
// panel p (tile column p, diagonal block D, tiles B_i = A[i][p] below it):
//   W_i = B_i D^-1           (i > p),
//   A[i][j] -= W_i B_j^T     (p < j <= i),
// and after the last panel the skeleton tiles hold S.  K_II^-1 is never
// formed; the multipliers W_i of every panel are kept for the interior
// recovery, which runs the panels backwards: u_p = -sum_{i > p} W_i^T u_i
// (the loads act on skeleton dofs only).  Padding rows stay decoupled, so
// their multipliers are zero.
//
// One workgroup of four waves per cell.  The lower tiles are distributed
// 2 x 2 cyclically (wave (wr, wc) holds the tiles (i, j) with i = wr and
// j = wc mod 2) and live in registers as FP64 MFMA 16x16x4 accumulator
// fragments: lane 16 g + c holds rows g, g + 4, g + 8, g + 12 of column c.
// Per panel: the owners of tile column p copy it to LDS (double buffered: one
// barrier per panel); every wave forms W_i for its tile rows on MFMA and
// applies the update to its trailing tiles on MFMA.  D^-1 is formed once per
// panel, ahead of time: the owner of the next diagonal tile updates that tile
// first and inverts it in its registers (Gauss-Jordan on pivot pairs, with row
// and row-group broadcasts) while the other waves run their updates, and
// leaves it in LDS for the next panel.
// The panels are taken in pairs and the register array moves up one tile row
// and column after each pair, so every register index is a compile-time
// constant while the panel loop is not unrolled.
//
// Outputs per cell: S packed lower row-major [nU(nU+1)/2]; W panel by panel
// (schur_w_count doubles), tile i of panel p at 256 (p (NT-1) - p (p-1)/2 +
// i - p - 1), entry (row r, column k) of the tile at 64 (k / 4) + 16 (k % 4)
// + r (the accumulator order, so that 64 lanes store and load it
// contiguously); and the skeleton diagonal of K (for the weights).
// Skeleton slots of Dirichlet nodes (slots without a global skeleton dof: the
// cell edges on clamped sides) are replaced by identity rows/columns (their
// Dirichlet values are zero).
#include "internal.h"
#include "wave_gj.h"

namespace lbddc {

typedef double dbl4s __attribute__((ext_vector_type(4)));

// The value of v in lane 16 g + k, for every lane of row g (16 lanes).
template <int k>
__device__ __forceinline__ double row_bcast(double v) {
  return __longlong_as_double(
      __builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x150 + k, 0xF, 0xF, false));
}

// The value of v in lane 16 q + c, for lane 16 g + c of every row g: the two
// halves of the wave exchanged, then the rows within each half.
template <int q>
__device__ __forceinline__ unsigned group_bcast32(unsigned t) {
  const auto h = __builtin_amdgcn_permlane32_swap(t, t, false, false);  // {low half twice, high half twice}
  const unsigned y = q < 2 ? h[0] : h[1];
  const auto r = __builtin_amdgcn_permlane16_swap(y, y, false, false);  // {even rows twice, odd rows twice}
  return (q & 1) ? r[1] : r[0];
}
template <int q>
__device__ __forceinline__ double group_bcast(double v) {
  const unsigned lo = group_bcast32<q>((unsigned)__double2loint(v));
  const unsigned hi = group_bcast32<q>((unsigned)__double2hiint(v));
  return __hiloint2double((int)hi, (int)lo);
}

// Gauss-Jordan elimination of the pivot pair K = {k, k + 1} (k even) on the
// 16 x 16 block held as one accumulator fragment (x[v] = D[g + 4v][c]): with
// Q = D[K][K]^-1 (2 x 2, by its adjugate),
//   D[K][K] <- Q,  D[K][c] <- Q D[K][c],  D[i][K] <- -D[i][K] Q,
//   D[i][c] <- D[i][c] - D[i][K] Q D[K][c]      (i, c not in K),
// the block form of the scalar rule of gj_inverse_wave (after all pairs D
// holds D^-1).  Rows k and k + 1 come from their row groups by the group
// broadcast, columns k and k + 1 from lanes k and k + 1 of each row by the row
// broadcast.  A pair costs one reciprocal: half the dependent steps of
// single pivots.  The block is SPD, so D[k][k] > 0 and det Q^-1 > 0; otherwise
// *bad is set and Q = I.
template <int k>
__device__ __forceinline__ void gj_pair(double (&x)[4], int g, int c, bool& bad) {
  constexpr int q0 = k & 3, vk = k >> 2;
  static_assert((k & 1) == 0, "pairs start at even pivots");
  const double r0 = group_bcast<q0>(x[vk]);      // D[k][c]
  const double r1 = group_bcast<q0 + 1>(x[vk]);  // D[k + 1][c]
  const double a = row_bcast<k>(r0), b = row_bcast<k + 1>(r0);
  const double b2 = row_bcast<k>(r1), d = row_bcast<k + 1>(r1);
  double c0[4], c1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    c0[v] = row_bcast<k>(x[v]);      // D[g + 4v][k]
    c1[v] = row_bcast<k + 1>(x[v]);  // D[g + 4v][k + 1]
  }
  const double det = fma(a, d, -b * b2);
  const bool ok = a > 0.0 && det > 0.0;
  bad = bad || !ok;
  const double id = recip_refined(ok ? det : 1.0);
  const double q00 = ok ? d * id : 1.0, q01 = ok ? -b * id : 0.0;
  const double q10 = ok ? -b2 * id : 0.0, q11 = ok ? a * id : 1.0;
  const double y0 = fma(q00, r0, q01 * r1), y1 = fma(q10, r0, q11 * r1);  // (Q D[K][c])
  const bool col0 = c == k, col1 = c == k + 1;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const bool row0 = v == vk && g == q0, row1 = v == vk && g == q0 + 1;
    const double z0 = -fma(c0[v], q00, c1[v] * q10), z1 = -fma(c0[v], q01, c1[v] * q11);
    const double off = fma(-c0[v], y0, fma(-c1[v], y1, x[v]));
    const double in0 = row0 ? q00 : row1 ? q10 : z0;
    const double in1 = row0 ? q01 : row1 ? q11 : z1;
    const double out = row0 ? y0 : row1 ? y1 : off;
    x[v] = col0 ? in0 : col1 ? in1 : out;
  }
}
// D^-1 in place by the first nk pivots (nk even; the rest are identity
// padding rows)
template <int k>
__device__ __forceinline__ void gj16(double (&x)[4], int nk, int g, int c, bool& bad) {
  if constexpr (k < 16) {
    if (k < nk) {
      gj_pair<k>(x, g, c, bad);
      gj16<k + 2>(x, nk, g, c, bad);
    }
  }
}

template <int P>
__global__ __launch_bounds__(256, 2) void k_schur(const double* __restrict__ K, const int* __restrict__ RU,
                                                  double* __restrict__ S, double* __restrict__ W,
                                                  double* __restrict__ diagK, int* __restrict__ flags) {
  constexpr int NN = (P + 1) * (P + 1), NI = 2 * (P - 1) * (P - 1), NU = 8 * P;
  constexpr int NIP = (NI + 15) / 16, NUT = (NU + 15) / 16, NT = NIP + NUT;
  constexpr int NA = (NT + 1) / 2, NQ = (NIP + 1) / 2, LDP = 17;
  constexpr int NPAIR = NN * (NN + 1) / 2, NSP = NU * (NU + 1) / 2;
  static_assert(NT <= 11 && NSP <= 2 * 16 * NT * LDP, "register tiles and S staging");
  const int cell = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: tile loops branch on scalars
  const int wr = wave >> 1, wc = wave & 1, g = lane >> 4, c = lane & 15;
  __shared__ double pb[2][16 * NT][LDP];
  __shared__ double dinv[2][16][LDP];     // D^-1 of the current and the next panel
  __shared__ unsigned char idr[16 * NT];  // 1: padding row or Dirichlet skeleton row (an identity row)
  for (int i = tid; i < 16 * NT; i += 256) {
    const int s = i - 16 * NIP;
    idr[i] = s < 0 ? i >= NI : (s >= NU || RU[(size_t)cell * NU + s] < 0);
  }
  __syncthreads();
  const double* Kc = K + (size_t)cell * NPAIR * 4;
  // Row 16 t + r of the padded order is dof node nb(t) + r / 2, component r % 2
  // (interior and skeleton offsets are even); rows r >= lim(t) of tile t are
  // padding.
  auto nb = [](int t) { return 8 * t + (t >= NIP ? NI / 2 - 8 * NIP : 0); };
  auto lim = [](int t) { return t == NIP - 1 ? NI - 16 * (NIP - 1) : t == NT - 1 ? NU - 16 * (NUT - 1) : 16; };
  // below the diagonal tiles the row node is never below the column node: the
  // entry of rows (node nb(i) + 2v + g / 2) and columns (node nb(j) + c / 2) is
  // a wave-uniform base plus a lane offset
  const int lane_off = 4 * (c >> 1) + 2 * (g & 1) + (c & 1), h = g >> 1;
  // every load of the wave's tiles first (padding entries read entry 0 and are
  // replaced below), so they are in flight together; the upper half of a
  // diagonal tile comes from the symmetric entry
  dbl4s T[NA][NA];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int ti = 2 * a + wr, tj = 2 * b + wc;
      if (ti < NT && tj <= ti) {
        const bool cpad = c >= lim(tj);
        const int lr = lim(ti);
        if (ti > tj) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int R = nb(ti) + 2 * v;
            const int e = 4 * (R * (R + 1) / 2 + nb(tj)) + h * 4 * (R + 1) + lane_off;
            T[a][b][v] = Kc[(cpad || g + 4 * v >= lr) ? 0 : e];
          }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int n1 = nb(ti) + 2 * v + h, n2 = nb(tj) + (c >> 1);
            const int e = n1 >= n2 ? 4 * (n1 * (n1 + 1) / 2 + n2) + 2 * (g & 1) + (c & 1)
                                   : 4 * (n2 * (n2 + 1) / 2 + n1) + 2 * (c & 1) + (g & 1);
            T[a][b][v] = Kc[(cpad || g + 4 * v >= lr) ? 0 : e];
          }
        }
      }
    }
  // identity rows and columns of padding and Dirichlet slots; the skeleton
  // diagonal of K
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int ti = 2 * a + wr, tj = 2 * b + wc;
      if (ti < NT && tj <= ti) {
        const bool fc = idr[16 * tj + c];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool dg = ti == tj && g + 4 * v == c;
          double val = T[a][b][v];
          if (ti == tj && ti >= NIP && dg && g + 4 * v < lim(ti))
            diagK[(size_t)cell * NU + 16 * (ti - NIP) + c] = idr[16 * ti + c] ? 0.0 : val;
          if (fc || idr[16 * ti + g + 4 * v]) val = dg ? 1.0 : 0.0;
          T[a][b][v] = val;
        }
      }
    }
  bool bad = false;
  double* Wc = W + (size_t)cell * schur_w_count(P);
  // D^-1 of panel p is formed once, by the owner of tile (p, p) as soon as the
  // tile is final (during panel p - 1; for panel 0 here), and read by every
  // wave from LDS after the panel's barrier
  if (wave == 0) {
    double y[4] = {T[0][0][0], T[0][0][1], T[0][0][2], T[0][0][3]};
    gj16<0>(y, NI, g, c, bad);
#pragma unroll
    for (int v = 0; v < 4; ++v) dinv[0][g + 4 * v][c] = y[v];
  }
  for (int q = 0; q < NQ; ++q) {
    // slot (a, b) holds tile (2 (a + q) + wr, 2 (b + q) + wc)
    for (int h = 0; h < 2; ++h) {
      const int p = 2 * q + h;
      if (p >= NIP) break;
      double(*pp)[LDP] = pb[p & 1];
      if (wc == h) {  // tile column p is slot column 0 of these waves
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const int ti = 2 * (a + q) + wr;
          if (ti >= p && ti < NT) {
#pragma unroll
            for (int v = 0; v < 4; ++v) pp[16 * ti + g + 4 * v][c] = T[a][0][v];
          }
        }
      }
      __syncthreads();
      double x[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) x[v] = dinv[p & 1][g + 4 * v][c];
      const int nk = NI - 16 * p;  // pivots of this panel (the rest padding: zero multipliers)
      const int wb = p * (NT - 1) - p * (p - 1) / 2 - p - 1;  // W tile of row ti: wb + ti
      // W_i^T = D^-1 B_i^T (D^-1 symmetric): lane 16 g + c gets W_i[c][g + 4v],
      // which is the A operand of W_i in the update
      auto multipliers = [&](int ti) {
        dbl4s wt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          if (4 * s < nk) wt = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s], pp[16 * ti + c][4 * s + g], wt, 0, 0, 0);
        if (wc == 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) Wc[256 * (wb + ti) + 64 * v + lane] = wt[v];
        }
        return wt;
      };
      auto update = [&](dbl4s& t, const dbl4s& wt, int tj) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
          if (4 * s < nk) t = __builtin_amdgcn_mfma_f64_16x16x4f64(-wt[s], pp[16 * tj + c][4 * s + g], t, 0, 0, 0);
      };
      // lookahead: tile (p + 1, p + 1) is slot (h, h) of wave (1 - h, 1 - h) and
      // the only tile of its row in the update; its owner finishes it first and
      // inverts it while the other waves update their tiles
      const bool ahead = p + 1 < NIP && wr == 1 - h && wc == 1 - h;
      if (ahead) {
        dbl4s t = T[0][0];
        if constexpr (NA > 1) if (h) t = T[1][1];
        update(t, multipliers(p + 1), p + 1);
        if constexpr (NA > 1) {
          if (h) T[1][1] = t; else T[0][0] = t;
        } else {
          T[0][0] = t;
        }
        double y[4] = {t[0], t[1], t[2], t[3]};
        gj16<0>(y, nk - 16, g, c, bad);
#pragma unroll
        for (int v = 0; v < 4; ++v) dinv[(p + 1) & 1][g + 4 * v][c] = y[v];
      }
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int ti = 2 * (a + q) + wr;
        if (ti > p && ti < NT && !(ahead && ti == p + 1)) {
          const dbl4s wt = multipliers(ti);
#pragma unroll
          for (int b = 0; b <= a; ++b) {
            const int tj = 2 * (b + q) + wc;
            if (tj > p && tj <= ti) update(T[a][b], wt, tj);
          }
        }
      }
    }
    if (q + 1 < NQ) {
#pragma unroll
      for (int a = 0; a + 1 < NA; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) T[a][b] = T[a + 1][b + 1];
    }
  }
  if (bad && lane == 0) atomicOr(flags, 8);
  __syncthreads();  // the panel buffers are free: stage S there
  double* sst = &pb[0][0][0];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int ti = 2 * (a + NQ - 1) + wr, tj = 2 * (b + NQ - 1) + wc;
      if (ti < NT && tj >= NIP && tj <= ti) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * (ti - NIP) + g + 4 * v, j = 16 * (tj - NIP) + c;
          if (i < NU && j <= i) sst[i * (i + 1) / 2 + j] = T[a][b][v];
        }
      }
    }
  __syncthreads();
  double* Sc = S + (size_t)cell * NSP;
  for (int i = tid; i < NSP; i += 256) Sc[i] = sst[i];
}

hipError_t launch_schur(Ctx* c) {
  dim3 grid(c->ncell), block(256);
#define SC_CASE(pp)                                                                                   \
  case pp:                                                                                            \
    hipLaunchKernelGGL(k_schur<pp>, grid, block, 0, c->stream, c->d_K, c->d_RU, c->d_S, c->d_W,       \
                       c->d_diagK, c->d_flags);                                                       \
    break;
  switch (c->p) {
    SC_CASE(2) SC_CASE(3) SC_CASE(4) SC_CASE(5) SC_CASE(6) SC_CASE(7) SC_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef SC_CASE
  return hipGetLastError();
}

}  // namespace lbddc
