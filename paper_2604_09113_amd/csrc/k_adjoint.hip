// Compliance J = f^T u and its gradient (A11).
//
// With K u = f and J = f^T u, dJ = 2 u^T df - u^T dK u: the adjoint state of
// the compliance is u itself, so the gradient reuses the PCG solution (no
// second solve).  Per cell, with the fast-assembly contraction of Alg. 4/5,
//   E = u^T K u = sum_{pairs P, s} Z[P, s] * Ihat[P, s],
//   Ihat[P, s] = sum_r Uhat[P, s, r] Itil[r],
//   Z[P, s]   = w_P sum_{i1 i2} theta[i1 i2, s] u[n1, i1] u[n2, i2]
// (w_P = 2 for n1 > n2, 1 on the diagonal node pairs), hence
//   H[r]        = dE/dItil[r]        = sum_{P, s} Uhat[P, s, r] Z[P, s]
//   G[i1 i2, s] = dE/dtheta[i1 i2,s] = sum_P w_P u u Ihat[P, s].
// k_adjoint computes both on MFMA with the same Uhat tiles as the assembly
// (Ihat as in the assembly; H as a second, transposed product).  k_chain
// applies the chain rule: dItil/dt through the derivative of the Lagrange
// interpolant of the reduced coordinates, and dtheta/dX through the
// pulled-back tensor Chat(J) and the Bernstein map.  The traction load depends
// on the loaded edge's control points through the curve Jacobian.
#include "internal.h"
#include "implicit_rule.h"

namespace lbddc {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// tiles16[i] = {group, first position in `sorted`, number of cells (<= 16), unused}
template <int KC, int RB>
__global__ __launch_bounds__(256) void k_adjoint(const double* const* __restrict__ utg,
                                                 const double* const* __restrict__ ut2g,
                                                 const double* __restrict__ theta, const double* __restrict__ itil,
                                                 const double* __restrict__ ucell, const int* __restrict__ sorted,
                                                 const int4* __restrict__ tiles, double* __restrict__ Hout, double* __restrict__ Gout, int ns,
                                                 int npair, int NPT, int itil_stride, int ndof) {
  extern __shared__ double lds[];
  const int4 td = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const bool valid = col < td.z;
  const int cell = sorted[td.y + (valid ? col : 0)];
  const int GW = 16 * ns * 4;
  double* Gw = lds + wave * GW;
  for (int i = lane; i < GW; i += 64) Gw[i] = 0.0;
  double b[KC];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) b[kc] = itil[(size_t)cell * itil_stride + 4 * kc + grp];
  dbl4 hacc[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) hacc[rb] = dbl4{0, 0, 0, 0};
  const double* uc = ucell + (size_t)cell * ndof;
  // theta in tile order ([tile][s][16 cells][4]): one step of the tile's 16
  // cells is one contiguous 512 B segment
  const double* th = theta + ((size_t)blockIdx.x * ns * 16 + col) * 4;
  // the group's Uhat tiles are read through pointers loaded from memory: say
  // that they are global memory (a flat load would also be counted by the
  // LDS/scalar counter, whose waits drain the prefetch)
  typedef const double __attribute__((address_space(1)))* GP;
  const GP ut = (GP)utg[td.x];
  const GP ut2 = (GP)ut2g[td.x];
  __syncthreads();
  // products w_P u[n1, i1] u[n2, i2] of the pair rows this lane feeds (4 pairs
  // x 4 components).  The node pairs are in triangular order, P = n1 (n1 + 1)
  // / 2 + n2 with n2 <= n1, so (n1, n2) is computed rather than loaded; the
  // displacement entries of a pair tile are requested a tile ahead (pair_load,
  // unconditional: pairs out of range read node 0 and get weight 0), and the
  // products are formed when the tile starts (pair_products)
  double ra[4][4], rw[4];
  auto pair_load = [&](int pt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int P = pt * 16 + 4 * grp + v;
      const bool ok = pt < NPT && P < npair && valid;
      const int Pc = ok ? P : 0;
      int n1 = (int)((sqrtf(8.0f * (float)Pc + 1.0f) - 1.0f) * 0.5f);
      if ((n1 + 1) * (n1 + 2) / 2 <= Pc) ++n1;
      if (n1 * (n1 + 1) / 2 > Pc) --n1;
      const int n2 = Pc - n1 * (n1 + 1) / 2;
      rw[v] = ok ? (n1 == n2 ? 1.0 : 2.0) : 0.0;
      ra[v][0] = uc[2 * n1];
      ra[v][1] = uc[2 * n1 + 1];
      ra[v][2] = uc[2 * n2];
      ra[v][3] = uc[2 * n2 + 1];
    }
  };
  auto pair_products = [&](double (&uu)[4][4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double w = rw[v], a0 = ra[v][0], a1 = ra[v][1], c0 = ra[v][2], c1 = ra[v][3];
      uu[v][0] = w * a0 * c0; uu[v][1] = w * a0 * c1; uu[v][2] = w * a1 * c0; uu[v][3] = w * a1 * c1;
    }
  };
  // Deep reduced bases (KC > 6) would need more than 256 registers with the
  // double-buffered operands, the second H chain and the displacement
  // prefetch of the shallow ones, and run one wave per SIMD; their lean form
  // (one H chain, the transposed tile loaded one step ahead, the pair
  // products formed at the start of each tile) keeps two.
  constexpr bool LEAN = KC > 6;
  dbl4 hacc2[LEAN ? 1 : RB];  // second accumulator chain of H (odd kk), added in a fixed order at the end
#pragma unroll
  for (int rb = 0; rb < (LEAN ? 1 : RB); ++rb) hacc2[rb] = dbl4{0, 0, 0, 0};
  auto base = [&](int& ptl, int& sl) {
    if (sl >= ns) {
      sl -= ns;
      ptl += 4;
    }
    if (ptl >= NPT) ptl = NPT - 1;
  };
  // MFMA operands of step s of pair tile pt; steps past the end belong to the
  // wave's next tile (pt + 4), and past the last tile to any valid address
  auto load_a = [&](int ptl, int sl, double (&a)[KC]) {
    base(ptl, sl);
    const GP ap = ut + ((size_t)ptl * ns + sl) * KC * 64 + lane;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) a[kc] = ap[kc * 64];
  };
  auto load_h = [&](int ptl, int sl, double (&a2)[RB][4]) {
    base(ptl, sl);
    const GP ap2 = ut2 + ((size_t)ptl * ns + sl) * RB * 4 * 64 + lane;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) a2[rb][kk] = ap2[(rb * 4 + kk) * 64];
  };
  double uu[4][4];
  // one step: Ihat of the 16 pairs x 16 cells on MFMA, H += Uhat2^T Z, G += u u Ihat
  auto step = [&](int s, const double (&a)[KC], const double (&a2)[RB][4]) {
    dbl4 d = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kc], b[kc], d, 0, 0, 0);
    const dbl4 t4 = *reinterpret_cast<const dbl4*>(th + (size_t)s * 64);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double z = t4[0] * uu[kk][0] + t4[1] * uu[kk][1] + t4[2] * uu[kk][2] + t4[3] * uu[kk][3];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (!LEAN && (kk & 1)) hacc2[LEAN ? 0 : rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[rb][kk], z, hacc2[LEAN ? 0 : rb], 0, 0, 0);
        else hacc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[rb][kk], z, hacc[rb], 0, 0, 0);
      }
    }
    // this lane's 4 pairs' contributions to the 4 components e; the 16-lane
    // groups then reduce-scatter so that group grp holds the total of e = grp:
    // across 32 lanes each lane keeps the half of e its group ends in, then
    // across 16 lanes the one component
    double g[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) g[e] = uu[0][e] * d[0] + uu[1][e] * d[1] + uu[2][e] * d[2] + uu[3][e] * d[3];
    const int hi = grp >> 1, lo = grp & 1;
    const double k0 = hi ? g[2] : g[0], k1 = hi ? g[3] : g[1];
    const double s0 = hi ? g[0] : g[2], s1 = hi ? g[1] : g[3];
    const double x0 = k0 + __shfl_xor(s0, 32), x1 = k1 + __shfl_xor(s1, 32);
    const double gm = (lo ? x1 : x0) + __shfl_xor(lo ? x0 : x1, 16);
    Gw[(col * ns + s) * 4 + grp] += gm;
  };
  if constexpr (LEAN) {
    double aA[KC], aB[KC], a2A[RB][4], a2B[RB][4];
    load_a(wave, 0, aA);
    load_h(wave, 0, a2A);
    load_a(wave, 1, aB);
    load_h(wave, 1, a2B);
    for (int pt = wave; pt < NPT; pt += 4) {
      pair_load(pt);
      pair_products(uu);
      for (int s = 0; s < ns; s += 2) {  // ns = 4 (q + 1)^2 is even
        step(s, aA, a2A);
        load_a(pt, s + 2, aA);
        load_h(pt, s + 2, a2A);
        step(s + 1, aB, a2B);
        load_a(pt, s + 3, aB);
        load_h(pt, s + 3, a2B);
      }
    }
  } else {
    // two operand sets take the steps in turn, each reloaded (two steps ahead)
    // right after the step that used it, without copies between them
    double aA[KC], a2A[RB][4], aB[KC], a2B[RB][4];
    load_a(wave, 0, aA);
    load_h(wave, 0, a2A);
    load_a(wave, 1, aB);
    load_h(wave, 1, a2B);
    pair_load(wave);
    pair_products(uu);
    pair_load(wave + 4);  // next pair tile: its loads overlap this tile's work
    for (int pt = wave; pt < NPT; pt += 4) {
      for (int s = 0; s < ns; s += 2) {  // ns = 4 (q + 1)^2 is even
        step(s, aA, a2A);
        load_a(pt, s + 2, aA);
        load_h(pt, s + 2, a2A);
        step(s + 1, aB, a2B);
        load_a(pt, s + 3, aB);
        load_h(pt, s + 3, a2B);
      }
      pair_products(uu);
      pair_load(pt + 8);
    }
  }
  if constexpr (!LEAN) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) hacc[rb] += hacc2[rb];
  }
  __syncthreads();
  // G: sum the four waves in a fixed order and write
  for (int i = threadIdx.x; i < GW; i += 256) {
    double v = lds[i] + lds[GW + i] + lds[2 * GW + i] + lds[3 * GW + i];
    const int c = i / (ns * 4), rest = i % (ns * 4);
    if (c < td.z) Gout[(size_t)sorted[td.y + c] * ns * 4 + rest] = v;
  }
  __syncthreads();
  // H: lane (grp, col) holds r = 16 rb + grp + 4 v
  const int HW = 16 * 16 * RB;
  double* Hw = lds + wave * HW;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) Hw[col * 16 * RB + 16 * rb + grp + 4 * v] = hacc[rb][v];
  __syncthreads();
  for (int i = threadIdx.x; i < HW; i += 256) {
    const double v = lds[i] + lds[HW + i] + lds[2 * HW + i] + lds[3 * HW + i];
    const int c = i / (16 * RB), r = i % (16 * RB);
    if (c < td.z && r < itil_stride) Hout[(size_t)sorted[td.y + c] * itil_stride + r] = v;
  }
}

struct ChainArgs {
  const double* ctrl; const int* family; const double* t; const double* tab; const int* fam_slot;
  const double* thr;  // [ncell][4] corner thresholds (Table 1 cells)
  const double* coeff[4];
  double lo[4], hi[4];
  int n_k[4], n_r[4], r[4], dim[4];
  int ncell, nx, ny, netx, m, nL, ns, itil_stride, p, ndof, nI;
  int edge;  // loaded side as a cell edge (0 left, 1 right, 2 bottom, 3 top)
  double lam, mu, rho;
  Tables T;
  const double* H; const double* G; const double* ucell; const double* trac;
  double* gcell;  // [ncell][(m+1)^2][2] per-cell dJ/dX (already with the minus sign and load term)
  double* gt;     // [ncell] dJ/dt
  const double* edge_br; const int* edge_nm;  // the material part of each edge (k_edge_roots)
  double* gmu;    // [ncell][4] dJ/dmu (k_load_mu adds the moving ends of the loaded edge)
};

// one thread per cell, templated on the map order so that the control points
// and their gradient stay in registers (the loop over the edge nodes runs to a
// fixed bound with the terms past the end masked)
template <int M>
__global__ __launch_bounds__(64) void k_chain(ChainArgs g) {
  constexpr int NP1 = (M + 1) * (M + 1);
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  const int ix = cell % g.nx, iy = cell / g.nx;
  // dJ/dt = -H . dItil/dt (cells of four-parameter families: k_chain_mu4)
  const int fam = g.family[cell];
  const int slot = g.fam_slot[fam];
  if (g.dim[slot] == 4) {
    g.gt[cell] = 0.0;
  } else {
    const double t = g.t[cell], lo = g.lo[slot], hi = g.hi[slot];
    const int nk = g.n_k[slot], R = g.r[slot], nr = g.n_r[slot];
    const double w = (hi - lo) / nk;
    int k = (int)floor((t - lo) / w);
    if (k > nk - 1) k = nk - 1;
    if (k < 0) k = 0;
    const double a = lo + k * w, b = lo + (k + 1) * w, h = b - a, tau = (t - a) / h;
    const double* nodes = g.tab + g.T.off_rnodes[slot];
    double dl[17];
    for (int j = 0; j <= R; ++j) {
      double s = 0.0;
      for (int l = 0; l <= R; ++l) {
        if (l == j) continue;
        double term = 1.0 / (nodes[j] - nodes[l]);
        for (int q = 0; q <= R; ++q)
          if (q != j && q != l) term *= (tau - nodes[q]) / (nodes[j] - nodes[q]);
        s += term;
      }
      dl[j] = s / h;
    }
    const double* cf = g.coeff[slot] + (size_t)k * (R + 1) * nr;
    double dE = 0.0;
    for (int r = 0; r < nr; ++r) {
      double s = 0.0;
      for (int j = 0; j <= R; ++j) s += dl[j] * cf[j * nr + r];
      dE += g.H[(size_t)cell * g.itil_stride + r] * (1.0 - g.rho) * s;
    }
    g.gt[cell] = -dE;
  }
  // dE/dX through Chat(J) at the interpolation points
  double X[NP1][2];
#pragma unroll
  for (int b = 0; b <= M; ++b)
#pragma unroll
    for (int a = 0; a <= M; ++a) {
      const double* P = g.ctrl + ((size_t)(M * iy + b) * g.netx + M * ix + a) * 2;
      X[b * (M + 1) + a][0] = P[0];
      X[b * (M + 1) + a][1] = P[1];
    }
  double gX[NP1][2];
#pragma unroll
  for (int a = 0; a < NP1; ++a) gX[a][0] = gX[a][1] = 0.0;
  const double lam = g.lam, mu = g.mu;
  for (int k3 = 0; k3 < g.nL; ++k3) {
    const double* dNp = g.tab + g.T.off_geo_dN + (size_t)k3 * NP1 * 2;
    double dN[NP1 * 2];
#pragma unroll
    for (int a = 0; a < 2 * NP1; ++a) dN[a] = dNp[a];
    double Gs[16];  // G[cell][s][i1 i2] of the point, s = (j1 2 + j2) nL + k3
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int e = 0; e < 4; ++e) Gs[4 * jj + e] = g.G[((size_t)cell * g.ns + jj * g.nL + k3) * 4 + e];
    double J[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
    for (int a = 0; a < NP1; ++a)
#pragma unroll
      for (int i = 0; i < 2; ++i) { J[i][0] += X[a][i] * dN[2 * a]; J[i][1] += X[a][i] * dN[2 * a + 1]; }
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double A[2][2] = {{J[1][1] / det, -J[0][1] / det}, {-J[1][0] / det, J[0][0] / det}};
    // forward-mode derivative of Chat along each unit perturbation E_pq of J
    double dEdJ[2][2];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
      for (int qq = 0; qq < 2; ++qq) {
        double dA[2][2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int mm = 0; mm < 2; ++mm) dA[j][mm] = -A[j][pp] * A[qq][mm];
        const double ddet = det * A[qq][pp];
        double acc = 0.0;
#pragma unroll
        for (int j1 = 0; j1 < 2; ++j1)
#pragma unroll
          for (int j2 = 0; j2 < 2; ++j2) {
            const double aa = A[j1][0] * A[j2][0] + A[j1][1] * A[j2][1];
            const double daa = dA[j1][0] * A[j2][0] + A[j1][0] * dA[j2][0] + dA[j1][1] * A[j2][1] + A[j1][1] * dA[j2][1];
#pragma unroll
            for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
              for (int i2 = 0; i2 < 2; ++i2) {
                const double v = lam * A[j1][i1] * A[j2][i2] + mu * ((i1 == i2 ? aa : 0.0) + A[j1][i2] * A[j2][i1]);
                const double dv = lam * (dA[j1][i1] * A[j2][i2] + A[j1][i1] * dA[j2][i2]) +
                                  mu * ((i1 == i2 ? daa : 0.0) + dA[j1][i2] * A[j2][i1] + A[j1][i2] * dA[j2][i1]);
                const double dC = ddet * v + det * dv;
                acc += Gs[4 * (j1 * 2 + j2) + 2 * i1 + i2] * dC;
              }
          }
        dEdJ[pp][qq] = acc;
      }
#pragma unroll
    for (int a = 0; a < NP1; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) gX[a][c] -= dEdJ[c][0] * dN[2 * a] + dEdJ[c][1] * dN[2 * a + 1];
  }
  // traction load on the loaded edge: 2 u . df/dX for the control points along
  // that edge
  const int e = g.edge;
  const bool on_side = (e == 0 && ix == 0) || (e == 1 && ix == g.nx - 1) || (e == 2 && iy == 0) ||
                       (e == 3 && iy == g.ny - 1);
  if (on_side) {
    const int nq = g.T.nq_load, p = g.p;
    const double* w = g.tab + g.T.off_load_w;
    const double* bl = g.tab + g.T.off_load_b;
    const double* dB = g.tab + g.T.off_load_dB;
    const int k_side = e < 2 ? iy : ix;
    const double t0 = g.trac[k_side * 2], t1 = g.trac[k_side * 2 + 1];
    const double* u = g.ucell + (size_t)cell * g.ndof;
    // the edge's control points, and their gradient, in arrays of their own:
    // every register index stays static (selects over the edge, no indexing
    // of X by a runtime value)
    double Pe[M + 1][2], gE[M + 1][2];
#pragma unroll
    for (int k = 0; k <= M; ++k)
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        Pe[k][cc] = e == 0 ? X[k * (M + 1)][cc] : e == 1 ? X[k * (M + 1) + M][cc] : e == 2 ? X[k][cc] : X[M * (M + 1) + k][cc];
        gE[k][cc] = 0.0;
      }
    // u . t at the edge nodes (permuted dofs: skeleton slots after the interior ones)
    double ut[17];
#pragma unroll
    for (int n = 0; n < 17; ++n) {
      const int nn = n <= p ? n : 0;
      const int node = (nn == 0) ? ((e == 1) ? 1 : (e == 3) ? 2 : 0)
                                 : (nn == p ? ((e == 0) ? 2 : (e == 2) ? 1 : 3) : 4 + e * (p - 1) + (nn - 1));
      ut[n] = u[g.nI + 2 * node] * t0 + u[g.nI + 2 * node + 1] * t1;
    }
    const int ce = cell * 4 + e, mat = g.edge_nm[2 * ce + 1];
    if (mat >= 0) {
      // a Table 1 cell: the load acts on the material part of the edge, whose
      // ends (parametric) do not move with the control points
      const double* xq = g.tab + g.T.off_load_x;
      const double* nodes = g.tab + g.T.off_edge_nodes;
      const double* bw = g.tab + g.T.off_edge_bw;
      const double* br = g.edge_br + (size_t)ce * kEdgeBreaks;
      const int nb = g.edge_nm[2 * ce];
      for (int iv = 0; iv + 1 < nb; ++iv) {
        if (!((mat >> iv) & 1)) continue;
        const double a = br[iv], b = br[iv + 1];
        for (int qd = 0; qd < nq; ++qd) {
          const double s = a + (b - a) * xq[qd];
          double dBs[5];
          bernstein_deriv_at(M, s, dBs);
          double d0 = 0, d1 = 0;
#pragma unroll
          for (int k = 0; k <= M; ++k) {
            d0 += dBs[k] * Pe[k][0];
            d1 += dBs[k] * Pe[k][1];
          }
          const double ds = sqrt(d0 * d0 + d1 * d1);
          double ub = 0.0;
#pragma unroll
          for (int n = 0; n < 17; ++n)
            if (n <= p) ub += ut[n] * gll_lagrange(nodes, bw, p, n, s);
          const double f = 2.0 * (b - a) * w[qd] * ub / ds;
#pragma unroll
          for (int k = 0; k <= M; ++k) {
            gE[k][0] += f * d0 * dBs[k];
            gE[k][1] += f * d1 * dBs[k];
          }
        }
      }
    } else {
      for (int qd = 0; qd < nq; ++qd) {
        double d0 = 0, d1 = 0;
#pragma unroll
        for (int k = 0; k <= M; ++k) {
          d0 += dB[k * nq + qd] * Pe[k][0];
          d1 += dB[k * nq + qd] * Pe[k][1];
        }
        const double ds = sqrt(d0 * d0 + d1 * d1);
        double ub = 0.0;
#pragma unroll
        for (int n = 0; n < 17; ++n)
          if (n <= p) ub += ut[n] * bl[n * nq + qd];
        const double f = 2.0 * w[qd] * ub / ds;
#pragma unroll
        for (int k = 0; k <= M; ++k) {
          gE[k][0] += f * d0 * dB[k * nq + qd];
          gE[k][1] += f * d1 * dB[k * nq + qd];
        }
      }
    }
#pragma unroll
    for (int k = 0; k <= M; ++k)
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        gX[k * (M + 1)][cc] += e == 0 ? gE[k][cc] : 0.0;
        gX[k * (M + 1) + M][cc] += e == 1 ? gE[k][cc] : 0.0;
        gX[k][cc] += e == 2 ? gE[k][cc] : 0.0;
        gX[M * (M + 1) + k][cc] += e == 3 ? gE[k][cc] : 0.0;
      }
  }
  double* out = g.gcell + (size_t)cell * NP1 * 2;
#pragma unroll
  for (int a = 0; a < NP1; ++a) { out[2 * a] = gX[a][0]; out[2 * a + 1] = gX[a][1]; }
}

// The traction on a Table 1 cell acts on the material part of the loaded
// edge, whose ends s* (roots of phi along the edge) move with the corner
// thresholds: phi = phi_0 - sum_k l_k mu_k gives ds*/dmu_k = l_k(s*) /
// (d phi / d s)(s*).  By the Leibniz rule the end adds
//   2 u . df/dmu_k = +-2 (sum_n (u_n . t) b_n(s*)) |x'(s*)| ds*/dmu_k
// (+ at the upper end of a material interval, - at the lower), added to
// dJ/dmu after k_chain_mu4.  One thread per cell.
__global__ __launch_bounds__(64) void k_load_mu(ChainArgs g) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  const int ix = cell % g.nx, iy = cell / g.nx, e = g.edge, m = g.m, p = g.p;
  const bool on_side = (e == 0 && ix == 0) || (e == 1 && ix == g.nx - 1) || (e == 2 && iy == 0) ||
                       (e == 3 && iy == g.ny - 1);
  if (!on_side) return;
  const int ce = cell * 4 + e, mat = g.edge_nm[2 * ce + 1];
  if (mat < 0) return;
  const int k_side = e < 2 ? iy : ix;
  const double t0 = g.trac[k_side * 2], t1 = g.trac[k_side * 2 + 1];
  const double* u = g.ucell + (size_t)cell * g.ndof;
  double P[5][2];
  for (int k = 0; k <= m; ++k) {
    const int a = e == 0 ? 0 : e == 1 ? m : k, b = e < 2 ? k : (e == 2 ? 0 : m);
    const double* Q = g.ctrl + ((size_t)(m * iy + b) * g.netx + m * ix + a) * 2;
    P[k][0] = Q[0];
    P[k][1] = Q[1];
  }
  rule::Cell c;
  c.fam = g.family[cell];
  for (int k = 0; k < 4; ++k) c.mu[k] = g.thr[(size_t)cell * 4 + k];
  const double* nodes = g.tab + g.T.off_edge_nodes;
  const double* bw = g.tab + g.T.off_edge_bw;
  const double* br = g.edge_br + (size_t)ce * kEdgeBreaks;
  const int nb = g.edge_nm[2 * ce];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int iv = 0; iv + 1 < nb; ++iv) {
    if (!((mat >> iv) & 1)) continue;
    for (int side = 0; side < 2; ++side) {
      const double s = br[iv + side];
      if (s <= 0.0 || s >= 1.0) continue;  // a corner of the cell: fixed
      // a break between two material intervals is the upper end of one and
      // the lower end of the other: the two terms cancel, and are skipped
      const int other = side ? iv + 1 : iv - 1;
      if (other >= 0 && ((mat >> other) & 1)) continue;
      const double x0 = e == 0 ? 0.0 : e == 1 ? 1.0 : s, y0 = e < 2 ? s : (e == 2 ? 0.0 : 1.0);
      double f, gx, gy;
      rule::phi_grad(c, x0, y0, f, gx, gy);
      const double dphi = e < 2 ? gy : gx;
      double dBs[5];
      bernstein_deriv_at(m, s, dBs);
      double d0 = 0, d1 = 0;
      for (int k = 0; k <= m; ++k) { d0 += dBs[k] * P[k][0]; d1 += dBs[k] * P[k][1]; }
      double ub = 0.0;
      for (int n = 0; n <= p; ++n) {
        const int node = (n == 0) ? ((e == 1) ? 1 : (e == 3) ? 2 : 0)
                                  : (n == p ? ((e == 0) ? 2 : (e == 2) ? 1 : 3) : 4 + e * (p - 1) + (n - 1));
        ub += (u[g.nI + 2 * node] * t0 + u[g.nI + 2 * node + 1] * t1) * gll_lagrange(nodes, bw, p, n, s);
      }
      const double v = (side ? 2.0 : -2.0) * ub * sqrt(d0 * d0 + d1 * d1) / dphi;
      acc[0] += v * (1.0 - x0) * (1.0 - y0);
      acc[1] += v * x0 * (1.0 - y0);
      acc[2] += v * (1.0 - x0) * y0;
      acc[3] += v * x0 * y0;
    }
  }
  for (int k = 0; k < 4; ++k) g.gmu[(size_t)cell * 4 + k] += acc[k];
}

// dJ/dmu_i = -(1 - rho) sum_nodes d/dmu_i [l_1 l_2 l_3 l_4](node) h(node),
// h(node) = sum_j H_j coeff[node][j], for the cells of four-parameter
// families (the derivative of the tensor Lagrange interpolant of Alg. 5; H =
// dE/dItil from the adjoint contraction), on the tiles of the cluster-sorted
// cell order.  For 64 cells of a tile, h = H coeff^T is a dense product on
// FP64 MFMA 16x16x4: wave w owns cells 16w..16w+15 (A operand: their H, n_r
// zero-padded to 48, in registers) and runs over 16-node blocks (B operand:
// the cluster's coefficients, a 64-node slab staged in LDS for all four
// waves); each result tile is weighted by the four derivative products of
// the cells' Lagrange bases and summed, and the 16 lanes of a row group then
// add their node columns with a butterfly.
struct ChainMu4Args {
  const double* mu; const double* tab;
  const double* coeff;
  double lo, hi;
  int n_k, n_r, r, off_rnodes;
  int itil_stride;
  double rho;
  const double* H;
  double* gmu;  // [ncell][4]
};

// R1 = r + 1 nodes per threshold, a compile-time constant (the node decode
// becomes multiplications).
template <int R1>
__global__ __launch_bounds__(256) void k_chain_mu4(ChainMu4Args g, const int* __restrict__ sorted,
                                                   const int4* __restrict__ tiles) {
  const int4 td = tiles[blockIdx.x];
  const int c0 = 64 * blockIdx.y;
  const int ncells = td.z - c0;
  if (ncells <= 0) return;  // uniform over the workgroup
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  constexpr int R = R1 - 1, nn = R1 * R1 * R1 * R1;
  const int nr = g.n_r;
  __shared__ double ell[64][4][9], dell[64][4][9];
  __shared__ double cf[64][49];
  {
    const int cl = t & 63;  // thread t: cell cl, coordinate w
    const int cell = sorted[td.y + c0 + (cl < ncells ? cl : 0)];
    double tau[4], hs[4];
    mdeim4_cluster(g.mu + (size_t)cell * 4, g.lo, g.hi, g.n_k, tau, hs);
    const double* x = g.tab + g.off_rnodes;
    for (int a = 0; a < R1; ++a) {
      ell[cl][w][a] = lag_value(x, R, a, tau[w]);
      dell[cl][w][a] = lag_deriv(x, R, a, tau[w]) / hs[w];
    }
  }
  double tau0[4], hs0[4];
  const int k = mdeim4_cluster(g.mu + (size_t)sorted[td.y] * 4, g.lo, g.hi, g.n_k, tau0, hs0);
  const double* C = g.coeff + (size_t)k * nn * nr;
  const int kq = lane >> 4, col = lane & 15;
  // A operand: H of cell 16 w + col at columns 4 ks + kq
  double hA[12];
  {
    const int cl = 16 * w + col;
    const int cell = sorted[td.y + c0 + (cl < ncells ? cl : 0)];
#pragma unroll
    for (int ks = 0; ks < 12; ++ks) {
      const int j = 4 * ks + kq;
      hA[ks] = j < nr ? g.H[(size_t)cell * g.itil_stride + j] : 0.0;
    }
  }
  double acc[4][4];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[v][i] = 0.0;
  for (int n0 = 0; n0 < nn; n0 += 64) {
    __syncthreads();
    for (int i = t; i < 64 * 48; i += 256) {
      const int jn = i / 48, j = i - jn * 48, n = n0 + jn;
      cf[jn][j] = (n < nn && j < nr) ? C[(size_t)n * nr + j] : 0.0;
    }
    __syncthreads();
    const int blocks = min(4, (nn - n0 + 15) >> 4);
    for (int nb = 0; nb < blocks; ++nb) {
      dbl4 d = dbl4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < 12; ++ks)
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(hA[ks], cf[16 * nb + col][4 * ks + kq], d, 0, 0, 0);
      // d[v]: cell 16 w + kq + 4 v, node n0 + 16 nb + col
      const int n = n0 + 16 * nb + col;
      if (n >= nn) continue;
      const int a1 = n % R1, q1 = n / R1, a2 = q1 % R1, q2 = q1 / R1, a3 = q2 % R1, a4 = q2 / R1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cl = 16 * w + kq + 4 * v;
        const double l1 = ell[cl][0][a1], l2 = ell[cl][1][a2], l3 = ell[cl][2][a3], l4 = ell[cl][3][a4];
        const double d1 = dell[cl][0][a1], d2 = dell[cl][1][a2], d3 = dell[cl][2][a3], d4 = dell[cl][3][a4];
        const double l12 = l1 * l2, l34 = l3 * l4;
        acc[v][0] += d1 * l2 * l34 * d[v];
        acc[v][1] += l1 * d2 * l34 * d[v];
        acc[v][2] += l12 * d3 * l4 * d[v];
        acc[v][3] += l12 * l3 * d4 * d[v];
      }
    }
  }
  // add the node columns of each row group: butterfly over the 16 lanes
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) acc[v][i] += __shfl_xor(acc[v][i], o);
  if (col == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int cl = 16 * w + kq + 4 * v;
      if (cl >= ncells) continue;
      const int cell = sorted[td.y + c0 + cl];
#pragma unroll
      for (int i = 0; i < 4; ++i) g.gmu[(size_t)cell * 4 + i] = -(1.0 - g.rho) * acc[v][i];
    }
  }
}

// net gradient: sum over the cells sharing each control point (fixed order)
__global__ void k_net_gather(const double* __restrict__ gcell, const int* __restrict__ ptr,
                             const int* __restrict__ own, double* __restrict__ gnet, int nnet) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnet) return;
  double a0 = 0.0, a1 = 0.0;
  for (int o = ptr[i]; o < ptr[i + 1]; ++o) { a0 += gcell[2 * (size_t)own[o]]; a1 += gcell[2 * (size_t)own[o] + 1]; }
  gnet[2 * i] = a0;
  gnet[2 * i + 1] = a1;
}

// J = f . x over the skeleton (tractions act on skeleton dofs only): partial
// sums per workgroup, then one workgroup adds them in order
__global__ void k_compliance_part(const double* __restrict__ f, const double* __restrict__ x, int N,
                                  double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256) s += f[i] * x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_compliance(const double* __restrict__ part, int n, double* __restrict__ J) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *J = sh[0];
}

template <int KC>
static void launch_adj(Ctx* c, const double* const* pu, const double* const* pu2, const int4* tiles, int ntiles,
                       const double* ucell, const double* theta16) {
  constexpr int RB = (4 * KC + 15) / 16;
  if (c->ns % 2 != 0) return;  // the kernel takes the steps of s in pairs (ns = 4 (q + 1)^2)
  const size_t lds = (size_t)4 * 16 * c->ns * 4 * sizeof(double);
  hipLaunchKernelGGL((k_adjoint<KC, RB>), dim3(ntiles), dim3(256), lds, c->stream, pu, pu2, theta16, c->d_itil,
                     ucell, c->d_sorted, tiles, c->d_H, c->d_G, c->ns, c->npair, c->NPT, 4 * c->KC,
                     c->ndof);
}

hipError_t launch_gradient(Ctx* c, int rhs) {
  hipError_t e;
  // 16-cell tiles per group, and the per-group tile pointers
  const int G = (int)c->group_counts.size();
  std::vector<int> tiles;
  std::vector<int> fam_first, fam_n;
  int start = 0, g0 = 0;
  for (size_t s = 0; s < c->fam_ids.size(); ++s) {
    fam_first.push_back((int)tiles.size() / 4);
    for (int k = 0; k < c->roms[c->fam_ids[s]].ncl; ++k, ++g0) {
      for (int o = 0; o < c->group_counts[g0]; o += 16) {
        tiles.push_back(g0);
        tiles.push_back(start + o);
        tiles.push_back(std::min(16, c->group_counts[g0] - o));
        tiles.push_back(0);
      }
      start += c->group_counts[g0];
    }
    fam_n.push_back((int)tiles.size() / 4 - fam_first.back());
  }
  std::vector<const void*> ptrs(2 * G);
  for (int g = 0; g < G; ++g) {
    const RomDev& R = c->roms[c->fam_ids[c->group_family[g]]];
    ptrs[g] = R.ut64[c->group_cluster[g]];
    ptrs[G + g] = R.ucol64[c->group_cluster[g]];
  }
  e = hipMemcpyAsync(c->d_adj_tiles, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(c->d_adj_ptrs, ptrs.data(), ptrs.size() * sizeof(void*), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  const double* const* pu = (const double* const*)c->d_adj_ptrs;
  hipEventRecord(c->ev[0], c->stream);
  e = launch_theta_tile16(c, reinterpret_cast<const int4*>(c->d_adj_tiles), (int)tiles.size() / 4, c->d_theta_t);
  if (e != hipSuccess) return e;
  for (size_t s = 0; s < c->fam_ids.size(); ++s) {
    if (fam_n[s] == 0) continue;
    const int4* tl = reinterpret_cast<const int4*>(c->d_adj_tiles) + fam_first[s];
    const double* uc = c->d_ucell + (size_t)rhs * c->ncell * c->ndof;
    const double* th = c->d_theta_t + (size_t)fam_first[s] * c->ns * 64;
    switch (c->roms[c->fam_ids[s]].KC) {
      case 1: launch_adj<1>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 2: launch_adj<2>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 3: launch_adj<3>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 4: launch_adj<4>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 5: launch_adj<5>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 6: launch_adj<6>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 7: launch_adj<7>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 8: launch_adj<8>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 9: launch_adj<9>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 10: launch_adj<10>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      case 11: launch_adj<11>(c, pu, pu + G, tl, fam_n[s], uc, th); break;
      default: return hipErrorInvalidValue;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipEventRecord(c->ev[1], c->stream);
  ChainArgs a = {};
  a.ctrl = c->d_ctrl; a.family = c->d_family; a.t = c->d_t; a.tab = c->d_tab; a.fam_slot = c->d_flags + 8;
  for (size_t s = 0; s < c->fam_ids.size() && s < 4; ++s) {
    const RomDev& R = c->roms[c->fam_ids[s]];
    a.coeff[s] = R.coeff; a.lo[s] = R.lo; a.hi[s] = R.hi; a.n_k[s] = R.n_k; a.n_r[s] = R.n_r; a.r[s] = R.r;
    a.dim[s] = R.dim;
  }
  a.ncell = c->ncell; a.nx = c->nx; a.ny = c->ny; a.netx = c->netx; a.m = c->m; a.nL = c->nL; a.ns = c->ns;
  a.itil_stride = 4 * c->KC; a.p = c->p; a.ndof = c->ndof; a.nI = c->nI;
  a.lam = c->E * c->nu / ((1 + c->nu) * (1 - 2 * c->nu));
  a.mu = c->E / (2 * (1 + c->nu));
  a.rho = c->rho; a.T = c->tab;
  a.H = c->d_H; a.G = c->d_G; a.ucell = c->d_ucell + (size_t)rhs * c->ncell * c->ndof;
  a.trac = c->d_trac + (size_t)rhs * c->n_side * 2;
  a.edge = c->load_edge;
  a.gcell = c->d_gcell; a.gt = c->d_gt + (size_t)rhs * c->ncell;
  a.thr = c->d_mu; a.edge_br = c->d_edge_br; a.edge_nm = c->d_edge_nm;
  a.gmu = c->d_gmu + (size_t)rhs * c->ncell * 4;
  switch (c->m) {
#define CHN(mm) case mm: hipLaunchKernelGGL(k_chain<mm>, dim3((c->ncell + 63) / 64), dim3(64), 0, c->stream, a); break;
    CHN(1) CHN(2) CHN(3) CHN(4)
#undef CHN
    default: return hipErrorInvalidValue;
  }
  if (c->any_dim4) {
    for (size_t sl = 0; sl < c->fam_ids.size() && sl < c->tile_fam_first.size(); ++sl) {
      const RomDev& R = c->roms[c->fam_ids[sl]];
      if (R.dim != 4 || c->tile_fam_n[sl] == 0) continue;
      if (R.r > 8 || R.n_r > 43) return hipErrorInvalidValue;
      ChainMu4Args b = {};
      b.mu = c->d_mu; b.tab = c->d_tab; b.coeff = R.coeff; b.lo = R.lo; b.hi = R.hi;
      b.n_k = R.n_k; b.n_r = R.n_r; b.r = R.r; b.off_rnodes = c->tab.off_rnodes[sl];
      b.itil_stride = 4 * c->KC; b.rho = c->rho; b.H = c->d_H;
      b.gmu = c->d_gmu + (size_t)rhs * c->ncell * 4;
      const int4* tl = reinterpret_cast<const int4*>(c->d_tiles) + c->tile_fam_first[sl];
      const dim3 grid(c->tile_fam_n[sl], 2);
      switch (R.r) {
#define CM4(rr) case rr: hipLaunchKernelGGL(k_chain_mu4<rr + 1>, grid, dim3(256), 0, c->stream, b, c->d_sorted, tl); break;
        CM4(1) CM4(2) CM4(3) CM4(4) CM4(5) CM4(6) CM4(7) CM4(8)
#undef CM4
        default: return hipErrorInvalidValue;
      }
    }
    hipLaunchKernelGGL(k_load_mu, dim3((c->ncell + 63) / 64), dim3(64), 0, c->stream, a);
  }
  const int nnet = c->netx * c->nety;
  hipLaunchKernelGGL(k_net_gather, dim3((nnet + 255) / 256), dim3(256), 0, c->stream, c->d_gcell, c->d_net_ptr,
                     c->d_net_own, c->d_gX + (size_t)rhs * nnet * 2, nnet);
  const int nparts = 256;
  hipLaunchKernelGGL(k_compliance_part, dim3(nparts), dim3(256), 0, c->stream, c->d_f + (size_t)rhs * c->NU,
                     c->d_x + (size_t)rhs * c->NU, c->NU, c->d_red);
  hipLaunchKernelGGL(k_compliance, dim3(1), dim3(256), 0, c->stream, c->d_red, nparts, c->d_J + rhs);
  return hipGetLastError();
}

}  // namespace lbddc

using namespace lbddc;

static lbddc_status grad_common(lbddc_ctx* x) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->solved) { c->err = "compliance_gradient: solve first"; return LBDDC_E_STATE; }
  hipSetDevice(c->device);
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  hipEventRecord(a, c->stream);
  for (int r = 0; r < c->nrhs; ++r) {
    hipError_t e = launch_gradient(c, r);
    if (e != hipSuccess) {
      c->err = std::string("compliance_gradient: ") + hipGetErrorString(e);
      return LBDDC_E_HIP;
    }
    if (r == 0) {
      hipEventSynchronize(c->ev[1]);
      float ms = 0;
      if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) c->phase_ms[11] = ms;
    }
  }
  hipEventRecord(b, c->stream);
  hipEventSynchronize(b);
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) == hipSuccess) c->phase_ms[10] = ms;
  hipEventDestroy(a);
  hipEventDestroy(b);
  return LBDDC_OK;
}

extern "C" lbddc_status lbddc_compliance_gradient(lbddc_ctx* x, double* J, double* dJ_dctrl, double* dJ_dt,
                                                  double* dJ_dmu) {
  lbddc_status s = grad_common(x);
  if (s != LBDDC_OK) return s;
  Ctx* c = &x->c;
  const size_t nnet = (size_t)c->netx * c->nety;
  hipError_t e = hipSuccess;
  if (J) e = hipMemcpyAsync(J, c->d_J, c->nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && dJ_dctrl)
    e = hipMemcpyAsync(dJ_dctrl, c->d_gX, c->nrhs * nnet * 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && dJ_dt)
    e = hipMemcpyAsync(dJ_dt, c->d_gt, (size_t)c->nrhs * c->ncell * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && dJ_dmu)
    e = hipMemcpyAsync(dJ_dmu, c->d_gmu, (size_t)c->nrhs * c->ncell * 4 * sizeof(double), hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->err = std::string("compliance_gradient copy: ") + hipGetErrorString(e);
    return LBDDC_E_HIP;
  }
  return LBDDC_OK;
}

extern "C" lbddc_status lbddc_compliance_gradient_device(lbddc_ctx* x, double* d_J, double* d_dJ_dctrl,
                                                         double* d_dJ_dt, double* d_dJ_dmu) {
  lbddc_status s = grad_common(x);
  if (s != LBDDC_OK) return s;
  Ctx* c = &x->c;
  const size_t nnet = (size_t)c->netx * c->nety;
  hipError_t e = hipSuccess;
  if (d_J) e = hipMemcpyAsync(d_J, c->d_J, c->nrhs * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && d_dJ_dctrl)
    e = hipMemcpyAsync(d_dJ_dctrl, c->d_gX, c->nrhs * nnet * 2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && d_dJ_dt)
    e = hipMemcpyAsync(d_dJ_dt, c->d_gt, (size_t)c->nrhs * c->ncell * sizeof(double), hipMemcpyDeviceToDevice,
                       c->stream);
  if (e == hipSuccess && d_dJ_dmu)
    e = hipMemcpyAsync(d_dJ_dmu, c->d_gmu, (size_t)c->nrhs * c->ncell * 4 * sizeof(double), hipMemcpyDeviceToDevice,
                       c->stream);
  if (e != hipSuccess) {
    c->err = std::string("compliance_gradient_device copy: ") + hipGetErrorString(e);
    return LBDDC_E_HIP;
  }
  return LBDDC_OK;
}
