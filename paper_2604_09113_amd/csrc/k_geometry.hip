// Per-cell geometry kernels.
//
// k_geometry (A1 + A2), one thread per (cell, interpolation point), templated
// on the map order:
//  * Jacobian of the Bernstein cell map at the (q+1)^2 interpolation points and
//    the pulled-back tensor Chat_{i1 j1 i2 j2} = det J A_{j1 m} C_{i1 m i2 n} A_{j2 n},
//    A = J^-1 (Sec. 2.2.1, pull-back of the elasticity tensor; Sec. 4.1, its
//    values at the interpolation points are the geometry coefficients), written
//    as theta[cell][s][i1 i2] with s = (j1*2 + j2)*nL + k3;
//  * det J > 0 check at the interpolation points and a Gauss sample;
//  * MDEIM online step (Alg. 5): cluster of t, Lagrange interpolation of the
//    fitted reduced coordinates, stabilised vector [(1-rho) I_r(t), rho]
//    (Alg. 4 folds the stabilisation into the last column).  For families
//    with four parameters per cell (the corner thresholds of Sec. 2.1.2) this
//    kernel finds the cluster and checks the box; k_mdeim4 evaluates the
//    tensor-product interpolant.
// k_constraints: edge-average and edge-moment rows of the coarse dofs
//  (Sec. 3.3.1) by Gauss quadrature along the physical edge.
// k_loads: consistent load of the traction on the loaded side (Sec. 2.2.1),
//  on the material part of the edge for Table 1 cells.
#include "internal.h"
#include "implicit_rule.h"

namespace lbddc {

struct GeoArgs {
  const double* ctrl; const int* family; const double* t; const double* thr; const double* tab;
  const int* fam_slot;        // family id -> slot (or -1); indexed by family id (< 64)
  const double* coeff[4];     // per slot [n_cl][(r+1)^dim][n_r]
  double lo[4], hi[4];
  int n_k[4], n_r[4], r[4], dim[4], group_base[4];
  int ncell, nx, netx, m, nL, ns, itil_stride;
  double lam, mu, rho;
  Tables T;
  double* theta; float* theta32; double* itil; float* itil32; int* group; int* flags;
};

template <int M>
__global__ __launch_bounds__(256) void k_geometry(GeoArgs g) {
  constexpr int NP1 = (M + 1) * (M + 1);
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int cell = tid / g.nL, k3 = tid - cell * g.nL;
  if (cell >= g.ncell) return;
  const int ix = cell % g.nx, iy = cell / g.nx;
  // the cell's control points, every load issued together
  double X[NP1][2];
#pragma unroll
  for (int b = 0; b <= M; ++b)
#pragma unroll
    for (int a = 0; a <= M; ++a) {
      const double* P = g.ctrl + ((size_t)(M * iy + b) * g.netx + M * ix + a) * 2;
      X[b * (M + 1) + a][0] = P[0];
      X[b * (M + 1) + a][1] = P[1];
    }
  auto jac = [&](const double* dN, double (&J)[2][2]) {
    double d[NP1][2];
#pragma unroll
    for (int a = 0; a < NP1; ++a) {
      d[a][0] = dN[2 * a];
      d[a][1] = dN[2 * a + 1];
    }
    J[0][0] = J[0][1] = J[1][0] = J[1][1] = 0.0;
#pragma unroll
    for (int a = 0; a < NP1; ++a)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        J[i][0] += X[a][i] * d[a][0];
        J[i][1] += X[a][i] * d[a][1];
      }
  };
  bool bad = false;
  // det J on the check sample, its points shared among the cell's threads
  for (int k = k3; k < g.T.nchk; k += g.nL) {
    double J[2][2];
    jac(g.tab + g.T.off_chk_dN + (size_t)k * NP1 * 2, J);
    if (!(J[0][0] * J[1][1] - J[0][1] * J[1][0] > 0.0)) bad = true;
  }
  const double lam = g.lam, mu = g.mu;
  {
    double J[2][2];
    jac(g.tab + g.T.off_geo_dN + (size_t)k3 * NP1 * 2, J);
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (!(det > 0.0)) bad = true;
    const double A[2][2] = {{J[1][1] / det, -J[0][1] / det}, {-J[1][0] / det, J[0][0] / det}};
#pragma unroll
    for (int j1 = 0; j1 < 2; ++j1)
#pragma unroll
      for (int j2 = 0; j2 < 2; ++j2) {
        const double aa = A[j1][0] * A[j2][0] + A[j1][1] * A[j2][1];
        const int s = (j1 * 2 + j2) * g.nL + k3;
#pragma unroll
        for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
          for (int i2 = 0; i2 < 2; ++i2) {
            // isotropic C_{i1 m i2 n} = lam d_{i1 m} d_{i2 n} + mu (d_{i1 i2} d_{mn} + d_{i1 n} d_{m i2})
            double v = lam * A[j1][i1] * A[j2][i2] + mu * ((i1 == i2 ? aa : 0.0) + A[j1][i2] * A[j2][i1]);
            v *= det;
            const size_t o = ((size_t)cell * g.ns + s) * 4 + 2 * i1 + i2;
            g.theta[o] = v;
            g.theta32[o] = (float)v;
          }
      }
  }
  if (bad) atomicOr(g.flags, 1);
  if (k3 != 0) return;
  // MDEIM online evaluation, by the cell's first thread
  const int fam = g.family[cell];
  const int slot = (fam >= 0 && fam < 64) ? g.fam_slot[fam] : -1;
  double* it = g.itil + (size_t)cell * g.itil_stride;
  float* it32 = g.itil32 + (size_t)cell * g.itil_stride;
  for (int r = 0; r < g.itil_stride; ++r) { it[r] = 0.0; it32[r] = 0.0f; }
  if (slot < 0) { atomicOr(g.flags, 4); g.group[cell] = 0; return; }
  if (g.dim[slot] == 4) {
    // cluster sum_i c_i n_k^i of the corner thresholds, first one fastest
    const double lo = g.lo[slot], hi = g.hi[slot];
    const int nk = g.n_k[slot];
    const double w = (hi - lo) / nk;
    int k = 0;
    for (int i = 3; i >= 0; --i) {
      const double v = g.thr[(size_t)cell * 4 + i];
      if (!(v >= lo && v <= hi)) { atomicOr(g.flags, 2); g.group[cell] = g.group_base[slot]; return; }
      int ci = (int)floor((v - lo) / w);
      if (ci > nk - 1) ci = nk - 1;
      if (ci < 0) ci = 0;
      k = k * nk + ci;
    }
    g.group[cell] = g.group_base[slot] + k;
    return;
  }
  const double t = g.t[cell], lo = g.lo[slot], hi = g.hi[slot];
  const int nk = g.n_k[slot], R = g.r[slot], nr = g.n_r[slot];
  if (!(t >= lo && t <= hi)) { atomicOr(g.flags, 2); g.group[cell] = g.group_base[slot]; return; }
  const double w = (hi - lo) / nk;
  int k = (int)floor((t - lo) / w);
  if (k > nk - 1) k = nk - 1;
  if (k < 0) k = 0;
  const double a = lo + k * w, b = lo + (k + 1) * w;
  const double tau = (t - a) / (b - a);
  const double* nodes = g.tab + g.T.off_rnodes[slot];
  // Lagrange basis at tau (degree R <= 16): fixed-size loops with the terms
  // past R masked, so the values stay in registers
  double nd[17], ell[17];
#pragma unroll
  for (int j = 0; j < 17; ++j) nd[j] = nodes[j <= R ? j : 0];
#pragma unroll
  for (int j = 0; j < 17; ++j) {
    double v = 1.0;
#pragma unroll
    for (int l = 0; l < 17; ++l)
      if (l != j && l <= R) v *= (tau - nd[l]) / (nd[j] - nd[l]);
    ell[j] = v;
  }
  const double* cf = g.coeff[slot] + (size_t)k * (R + 1) * nr;
  for (int r = 0; r < nr; ++r) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 17; ++j)
      if (j <= R) s += ell[j] * cf[j * nr + r];
    s *= (1.0 - g.rho);
    it[r] = s;
    it32[r] = (float)s;
  }
  it[nr] = g.rho;
  it32[nr] = (float)g.rho;
  g.group[cell] = g.group_base[slot] + k;
}

// MDEIM online step for the cells of four-parameter families (Alg. 5 with a
// tensor fitting grid, Sec. 4.2.3), on the tiles of the cluster-sorted cell
// order that the contraction uses (every cell of a tile is in the same
// cluster).  For 64 cells of a tile it is the dense product
//   Itil[cell][j] = (1 - rho) sum_nodes W[cell][node] coeff[node][j],
//   W[cell][node] = l_1(a_1) l_2(a_2) l_3(a_3) l_4(a_4)   (Lagrange bases at the cell's tau),
// over the (r+1)^4 nodes (node a_1 + (r+1)(a_2 + (r+1)(a_3 + (r+1) a_4))), on
// FP64 MFMA 16x16x4: wave w owns cells 16w..16w+15 and the three 16-column
// blocks of j (n_r <= 43, zero-padded to 48), forms its A operand (16 cells x
// 4 nodes of W) from the per-cell bases in LDS, and reads the B operand (4
// nodes x 16 columns) from a 64-node slab of the cluster's coefficients
// staged in LDS for all four waves.
typedef double dbl4g __attribute__((ext_vector_type(4)));

struct Mdeim4Args {
  const double* mu; const double* tab;
  const double* coeff;
  double lo, hi;
  int n_k, n_r, r, off_rnodes;
  int itil_stride;
  double rho;
  double* itil; float* itil32;
};

// R1 = r + 1 nodes per threshold, a compile-time constant so that the node
// decode n -> (a1, a2, a3, a4) is multiplications, not integer divisions.
template <int R1>
__global__ __launch_bounds__(256) void k_mdeim4(Mdeim4Args g, const int* __restrict__ sorted,
                                                const int4* __restrict__ tiles) {
  const int4 td = tiles[blockIdx.x];
  const int c0 = 64 * blockIdx.y;
  const int ncells = td.z - c0;
  if (ncells <= 0) return;  // uniform over the workgroup
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  constexpr int R = R1 - 1, nn = R1 * R1 * R1 * R1;
  const int nr = g.n_r;
  __shared__ double ell[64][4][9];
  __shared__ double cf[64][49];
  {
    const int cl = t & 63;  // thread t: cell cl, coordinate w
    const int cell = sorted[td.y + c0 + (cl < ncells ? cl : 0)];
    double tau[4], hs[4];
    mdeim4_cluster(g.mu + (size_t)cell * 4, g.lo, g.hi, g.n_k, tau, hs);
    const double* x = g.tab + g.off_rnodes;
    for (int a = 0; a < R1; ++a) ell[cl][w][a] = lag_value(x, R, a, tau[w]);
  }
  double tau0[4], hs0[4];
  const int k = mdeim4_cluster(g.mu + (size_t)sorted[td.y] * 4, g.lo, g.hi, g.n_k, tau0, hs0);
  const double* C = g.coeff + (size_t)k * nn * nr;
  const int row = 16 * w + (lane & 15), kq = lane >> 4, col = lane & 15;
  dbl4g acc[3];
#pragma unroll
  for (int rb = 0; rb < 3; ++rb) acc[rb] = dbl4g{0, 0, 0, 0};
  for (int n0 = 0; n0 < nn; n0 += 64) {
    __syncthreads();
    for (int i = t; i < 64 * 48; i += 256) {
      const int jn = i / 48, j = i - jn * 48, n = n0 + jn;
      cf[jn][j] = (n < nn && j < nr) ? C[(size_t)n * nr + j] : 0.0;
    }
    __syncthreads();
    const int steps = min(16, (nn - n0 + 3) >> 2);
    for (int st = 0; st < steps; ++st) {
      const int jn = 4 * st + kq, n = n0 + jn;
      double a = 0.0;
      if (n < nn) {
        const int a1 = n % R1, q1 = n / R1, a2 = q1 % R1, q2 = q1 / R1, a3 = q2 % R1, a4 = q2 / R1;
        a = ell[row][0][a1] * ell[row][1][a2] * ell[row][2][a3] * ell[row][3][a4];
      }
#pragma unroll
      for (int rb = 0; rb < 3; ++rb) acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, cf[jn][16 * rb + col], acc[rb], 0, 0, 0);
    }
  }
  // lane (g, c) holds cells 16 w + g + 4 v, columns 16 rb + c
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int cl = 16 * w + kq + 4 * v;
    if (cl >= ncells) continue;
    const int cell = sorted[td.y + c0 + cl];
    double* it = g.itil + (size_t)cell * g.itil_stride;
    float* it32 = g.itil32 + (size_t)cell * g.itil_stride;
#pragma unroll
    for (int rb = 0; rb < 3; ++rb) {
      const int j = 16 * rb + col;
      if (j < nr) {
        const double val = (1.0 - g.rho) * acc[rb][v];
        it[j] = val;
        it32[j] = (float)val;
      } else if (j == nr) {
        it[j] = g.rho;
        it32[j] = (float)g.rho;
      }
    }
  }
}

hipError_t launch_mdeim4(Ctx* c, int slot, const int* d_tiles, int first, int n) {
  const RomDev& R = c->roms[c->fam_ids[slot]];
  if (R.dim != 4 || n == 0) return hipSuccess;
  if (R.r > 8 || R.n_r > 43) return hipErrorInvalidValue;  // LDS bases hold r <= 8, four column quarters of <= 11
  Mdeim4Args a = {};
  a.mu = c->d_mu; a.tab = c->d_tab; a.coeff = R.coeff; a.lo = R.lo; a.hi = R.hi;
  a.n_k = R.n_k; a.n_r = R.n_r; a.r = R.r; a.off_rnodes = c->tab.off_rnodes[slot];
  a.itil_stride = 4 * c->KC; a.rho = c->rho; a.itil = c->d_itil; a.itil32 = c->d_itil32;
  const int4* tl = reinterpret_cast<const int4*>(d_tiles) + first;
  switch (R.r) {
#define MD4(rr) case rr: hipLaunchKernelGGL(k_mdeim4<rr + 1>, dim3(n, 2), dim3(256), 0, c->stream, a, c->d_sorted, tl); break;
    MD4(1) MD4(2) MD4(3) MD4(4) MD4(5) MD4(6) MD4(7) MD4(8)
#undef MD4
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Edge rows: for edge e of a cell, averages int_e u_c ds and moment
// int_e (x2 - xbar2) u1 + (xbar1 - x1) u2 ds over the p+1 edge nodes, xbar the
// image of the parametric midpoint; Gauss 2p+2 points along the physical edge.
struct ConsArgs {
  const double* ctrl; const double* tab; Tables T;
  int ncell, nx, netx, m, p, nce;
  double* cons;  // [ncell][4][nce][p+1][2]
  const int* family; const double* mu; const int* fam_slot; int dim[4];
  int* flags;
  double* edge_br; int* edge_nm;  // the material part of each edge
};

__device__ inline void edge_points(const double* ctrl, int netx, int m, int ix, int iy, int e, double P[5][2]) {
  for (int k = 0; k <= m; ++k) {
    int a, b;
    if (e == 0) { a = 0; b = k; }        // left   (xi1 = 0)
    else if (e == 1) { a = m; b = k; }   // right  (xi1 = 1)
    else if (e == 2) { a = k; b = 0; }   // bottom (xi2 = 0)
    else { a = k; b = m; }               // top    (xi2 = 1)
    const double* Q = ctrl + ((size_t)(m * iy + b) * netx + m * ix + a) * 2;
    P[k][0] = Q[0];
    P[k][1] = Q[1];
  }
}

// Root sink of the constraint rows: the face-root search of the implicit rule
// emits no points.
struct NoPoints {
  int err;
  __device__ void emit(double, double, double) {}
};

// The material part of each cell edge of a Table 1 level set: the sorted
// breaks (the ends and the roots of phi along the edge, found by the implicit
// rule's interval-checked search) and the mask of the intervals between them
// where phi < 0.  One lane per (cell, edge); edges of the one-parameter
// families get the mask -1 (the whole edge).
__global__ __launch_bounds__(64) void k_edge_roots(ConsArgs g) {
  const int ce = blockIdx.x * blockDim.x + threadIdx.x;
  if (ce >= g.ncell * 4) return;
  const int cell = ce >> 2, e = ce & 3;
  const int fam = g.family[cell];
  const int slot = (fam >= 0 && fam < 64) ? g.fam_slot[fam] : -1;
  int nb = 0, mat = -1;
  if (slot >= 0 && g.dim[slot] == 4) {
    rule::Cell c;
    c.fam = fam;
    for (int k = 0; k < 4; ++k) c.mu[k] = g.mu[(size_t)cell * 4 + k];
    // the edge as a face of the unit cell: xi_k = face, running coordinate in [0, 1]
    const int k = e < 2 ? 0 : 1;
    const double face = (e == 1 || e == 3) ? 1.0 : 0.0;
    double br[kEdgeBreaks];
    br[nb++] = 0.0;
    br[nb++] = 1.0;
    NoPoints sink{0};
    rule::face_roots(c, k, face, 0.0, 1.0, br, nb, kEdgeBreaks, sink);
    if (sink.err) atomicOr(g.flags, 1 << 7);
    for (int i = 1; i < nb; ++i) {
      const double v = br[i];
      int j = i - 1;
      while (j >= 0 && br[j] > v) {
        br[j + 1] = br[j];
        --j;
      }
      br[j + 1] = v;
    }
    mat = 0;
    for (int i = 0; i + 1 < nb; ++i) {
      const double mid = 0.5 * (br[i] + br[i + 1]);
      if (br[i + 1] > br[i] && rule::phi(c, k == 0 ? face : mid, k == 0 ? mid : face) < 0.0) mat |= 1 << i;
    }
    for (int i = 0; i < nb; ++i) g.edge_br[(size_t)ce * kEdgeBreaks + i] = br[i];
  }
  g.edge_nm[2 * ce] = nb;
  g.edge_nm[2 * ce + 1] = mat;
}

// The coarse rows of one node of one cell edge, one thread per (cell, edge,
// edge node).  The edge integrals run over the whole physical edge for the
// one-parameter families, and over the material part of the edge (phi_0 < mu)
// for the level sets of Table 1: on a lattice that meets the trimmed
// compatibility of Sec. 2.1.3 both cells sharing an edge see the same
// material part, so the averages and moments stay one functional of the
// shared edge values.  Every material interval gets the 2p+2 point Gauss rule.
__global__ __launch_bounds__(256) void k_constraints(ConsArgs g) {
  const int p = g.p, m = g.m, nq = g.T.nq_edge;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.ncell * 4 * (p + 1)) return;
  const int n = id % (p + 1), ce = id / (p + 1), cell = ce >> 2, e = ce & 3;
  const int ix = cell % g.nx, iy = cell / g.nx;
  double P[5][2];
  edge_points(g.ctrl, g.netx, m, ix, iy, e, P);
  const double* w = g.tab + g.T.off_edge_w;
  const double* Bm = g.tab + g.T.off_mid_B;
  double xb0 = 0, xb1 = 0;
  for (int k = 0; k <= m; ++k) { xb0 += Bm[k] * P[k][0]; xb1 += Bm[k] * P[k][1]; }
  double avg = 0, m0 = 0, m1 = 0;
  const int nb = g.edge_nm[2 * ce], mat = g.edge_nm[2 * ce + 1];
  if (mat >= 0) {
    const double* xq = g.tab + g.T.off_edge_x;
    const double* nodes = g.tab + g.T.off_edge_nodes;
    const double bw = g.tab[g.T.off_edge_bw + n];
    const double* br = g.edge_br + (size_t)ce * kEdgeBreaks;
    for (int iv = 0; iv + 1 < nb; ++iv) {
      if (!((mat >> iv) & 1)) continue;  // void interval
      const double a = br[iv], b = br[iv + 1];
      for (int qd = 0; qd < nq; ++qd) {
        const double xi = a + (b - a) * xq[qd];
        // GLL Lagrange polynomial of node n in barycentric form
        double bn = bw;
        for (int l = 0; l <= p; ++l)
          if (l != n) bn *= xi - nodes[l];
        // the edge curve and its tangent: Bernstein polynomials of degree m at xi
        double pw[5], pw1[5];  // xi^j and (1 - xi)^j
        pw[0] = pw1[0] = 1.0;
        for (int j = 1; j <= m; ++j) { pw[j] = pw[j - 1] * xi; pw1[j] = pw1[j - 1] * (1.0 - xi); }
        double x0 = 0, x1 = 0, d0 = 0, d1 = 0, binom = 1.0;
        for (int kk = 0; kk <= m; ++kk) {
          if (kk > 0) binom = binom * (m - kk + 1) / kk;
          const double bv = binom * pw[kk] * pw1[m - kk];
          const double dl = kk > 0 ? kk * binom * pw[kk - 1] * pw1[m - kk] : 0.0;
          const double dr = kk < m ? (m - kk) * binom * pw[kk] * pw1[m - kk - 1] : 0.0;
          x0 += bv * P[kk][0]; x1 += bv * P[kk][1];
          d0 += (dl - dr) * P[kk][0]; d1 += (dl - dr) * P[kk][1];
        }
        const double ws = (b - a) * w[qd] * sqrt(d0 * d0 + d1 * d1) * bn;
        avg += ws;
        m0 += ws * (x1 - xb1);
        m1 += ws * (xb0 - x0);
      }
    }
  } else {
    const double* bl = g.tab + g.T.off_edge_b;
    const double* B = g.tab + g.T.off_edge_B;
    const double* dB = g.tab + g.T.off_edge_dB;
    for (int qd = 0; qd < nq; ++qd) {
      double x0 = 0, x1 = 0, d0 = 0, d1 = 0;
      for (int kk = 0; kk <= m; ++kk) {
        x0 += B[kk * nq + qd] * P[kk][0]; x1 += B[kk * nq + qd] * P[kk][1];
        d0 += dB[kk * nq + qd] * P[kk][0]; d1 += dB[kk * nq + qd] * P[kk][1];
      }
      const double ws = w[qd] * sqrt(d0 * d0 + d1 * d1) * bl[n * nq + qd];
      avg += ws;
      m0 += ws * (x1 - xb1);
      m1 += ws * (xb0 - x0);
    }
  }
  double* out = g.cons + (size_t)ce * g.nce * (p + 1) * 2;
  out[(0 * (p + 1) + n) * 2 + 0] = avg;
  out[(0 * (p + 1) + n) * 2 + 1] = 0.0;
  out[(1 * (p + 1) + n) * 2 + 0] = 0.0;
  out[(1 * (p + 1) + n) * 2 + 1] = avg;
  if (g.nce > 2) {
    out[(2 * (p + 1) + n) * 2 + 0] = m0;
    out[(2 * (p + 1) + n) * 2 + 1] = m1;
  }
}

// Traction on the cell edges along the loaded side:
// f[node][c] = t_c int b_node |x'| dxi over the edge.
struct LoadArgs {
  const double* ctrl; const double* tab; const double* trac; Tables T;
  int ncell, nx, ny, netx, m, p, nU, nrhs;
  int edge, n_side;  // loaded side as a cell edge (0 left, 1 right, 2 bottom, 3 top)
  double* load;  // [nrhs][ncell][nU]
  const double* edge_br; const int* edge_nm;  // the material part of each edge (k_edge_roots)
};

// Skeleton node slot of node n (0..p, increasing running coordinate) of edge e:
// the corners BL 0, BR 1, TL 2, TR 3, then the interior nodes of the left,
// right, bottom and top edges, p - 1 each.
__device__ __forceinline__ int edge_node_slot(int e, int n, int p) {
  if (n == 0) return (e == 1) ? 1 : (e == 3) ? 2 : 0;
  if (n == p) return (e == 0) ? 2 : (e == 2) ? 1 : 3;
  return 4 + e * (p - 1) + (n - 1);
}

// one 64-lane workgroup per (cell, load case), lane l writing slot l (nU <= 64,
// coalesced): zero, or on the loaded edge the load of its node and component.
__global__ __launch_bounds__(64) void k_loads(LoadArgs g) {
  const int cell = blockIdx.x, rhs = blockIdx.y, l = threadIdx.x, p = g.p, e = g.edge;
  const int ix = cell % g.nx, iy = cell / g.nx;
  if (l >= g.nU) return;
  double* out = g.load + ((size_t)rhs * g.ncell + cell) * g.nU;
  const int node = l >> 1, comp = l & 1;
  int n = -1;
  for (int k = 0; k <= p; ++k)
    if (edge_node_slot(e, k, p) == node) n = k;
  const bool on_side = (e == 0 && ix == 0) || (e == 1 && ix == g.nx - 1) || (e == 2 && iy == 0) ||
                       (e == 3 && iy == g.ny - 1);
  if (!on_side || n < 0) {
    out[l] = 0.0;
    return;
  }
  const int k_side = e < 2 ? iy : ix;
  double P[5][2];
  edge_points(g.ctrl, g.netx, g.m, ix, iy, e, P);
  const int nq = g.T.nq_load;
  const double* w = g.tab + g.T.off_load_w;
  const double* bl = g.tab + g.T.off_load_b;
  const double* dB = g.tab + g.T.off_load_dB;
  const double tc = g.trac[((size_t)rhs * g.n_side + k_side) * 2 + comp];
  double f = 0;
  const int ce = cell * 4 + e, mat = g.edge_nm[2 * ce + 1];
  if (mat >= 0) {
    // a Table 1 cell: the traction acts on the material part of the edge
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
        bernstein_deriv_at(g.m, s, dBs);
        double d0 = 0, d1 = 0;
        for (int k = 0; k <= g.m; ++k) { d0 += dBs[k] * P[k][0]; d1 += dBs[k] * P[k][1]; }
        f += (b - a) * w[qd] * gll_lagrange(nodes, bw, p, n, s) * sqrt(d0 * d0 + d1 * d1);
      }
    }
  } else {
    for (int qd = 0; qd < nq; ++qd) {
      double d0 = 0, d1 = 0;
      for (int k = 0; k <= g.m; ++k) { d0 += dB[k * nq + qd] * P[k][0]; d1 += dB[k * nq + qd] * P[k][1]; }
      f += w[qd] * bl[n * nq + qd] * sqrt(d0 * d0 + d1 * d1);
    }
  }
  out[l] = f * tc;
}

hipError_t launch_geometry(Ctx* c) {
  GeoArgs g = {};
  g.ctrl = c->d_ctrl; g.family = c->d_family; g.t = c->d_t; g.thr = c->d_mu; g.tab = c->d_tab;
  static_assert(sizeof(int) == 4, "");
  g.fam_slot = c->d_flags + 8;  // family -> slot table lives after the flags
  int base = 0;
  for (size_t s = 0; s < c->fam_ids.size() && s < 4; ++s) {
    const RomDev& R = c->roms[c->fam_ids[s]];
    g.coeff[s] = R.coeff; g.lo[s] = R.lo; g.hi[s] = R.hi; g.n_k[s] = R.n_k; g.n_r[s] = R.n_r; g.r[s] = R.r;
    g.dim[s] = R.dim;
    g.group_base[s] = base;
    base += R.ncl;
  }
  g.ncell = c->ncell; g.nx = c->nx; g.netx = c->netx; g.m = c->m; g.nL = c->nL; g.ns = c->ns;
  g.itil_stride = 4 * c->KC;
  g.lam = c->E * c->nu / ((1 + c->nu) * (1 - 2 * c->nu));
  g.mu = c->E / (2 * (1 + c->nu));
  g.rho = c->rho; g.T = c->tab;
  g.theta = c->d_theta; g.theta32 = c->d_theta32; g.itil = c->d_itil; g.itil32 = c->d_itil32;
  g.group = c->d_cluster; g.flags = c->d_flags;
  const int nth = c->ncell * c->nL;  // one thread per (cell, interpolation point)
  switch (c->m) {
#define GEO(mm) case mm: hipLaunchKernelGGL(k_geometry<mm>, dim3((nth + 255) / 256), dim3(256), 0, c->stream, g); break;
    GEO(1) GEO(2) GEO(3) GEO(4)
#undef GEO
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_constraints_loads(Ctx* c, hipStream_t st) {
  ConsArgs a = {c->d_ctrl, c->d_tab, c->tab, c->ncell, c->nx, c->netx, c->m, c->p, c->nce, c->d_cons};
  a.family = c->d_family; a.mu = c->d_mu; a.fam_slot = c->d_flags + 8; a.flags = c->d_flags;
  a.edge_br = c->d_edge_br; a.edge_nm = c->d_edge_nm;
  for (size_t s = 0; s < c->fam_ids.size() && s < 4; ++s) a.dim[s] = c->roms[c->fam_ids[s]].dim;
  const int nedge = c->ncell * 4, nth = nedge * (c->p + 1);
  hipLaunchKernelGGL(k_edge_roots, dim3((nedge + 63) / 64), dim3(64), 0, st, a);
  hipLaunchKernelGGL(k_constraints, dim3((nth + 255) / 256), dim3(256), 0, st, a);
  LoadArgs l = {c->d_ctrl, c->d_tab, c->d_trac, c->tab, c->ncell, c->nx, c->ny, c->netx, c->m, c->p, c->nU, c->nrhs,
                c->load_edge, c->n_side, c->d_load};
  l.edge_br = c->d_edge_br; l.edge_nm = c->d_edge_nm;
  if (c->nU > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_loads, dim3(c->ncell, c->nrhs), dim3(64), 0, st, l);
  return hipGetLastError();
}

}  // namespace lbddc
