// Internal declarations of the lbddc library: the context, device buffers and
// the kernel launchers.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/lbddc.h"

namespace lbddc {

constexpr int kMaxP = 10;
constexpr int kMaxKC = 11;  // reduced basis + stabilisation column padded to 4*KC <= 44
constexpr int kMaxDevices = 64;
// load cases solved together by the block PCG (more are taken in blocks)
constexpr int kBlockRhs = 8;
constexpr int kEdgeBreaks = 16;  // breaks of one cell edge's material part (ends and roots)

// Doubles per cell of the interior elimination multipliers W of the local
// Schur complement: interior and skeleton dofs each padded to 16-row tiles
// (NIP and NUT of them), 256 doubles for every tile below each interior
// panel.
__host__ __device__ constexpr int schur_w_count(int p) {
  return 256 * (((2 * (p - 1) * (p - 1) + 15) / 16) * (((2 * (p - 1) * (p - 1) + 15) / 16) + (8 * p + 15) / 16 - 1) -
                ((2 * (p - 1) * (p - 1) + 15) / 16) * (((2 * (p - 1) * (p - 1) + 15) / 16) - 1) / 2);
}
// bytes of the static device scratch of lbddc_assemble_fp32_noalloc
constexpr size_t kNoAllocScratchBytes = 48u << 20;

// ---------------------------------------------------------------------------
// Host numerics (host_math.cpp): Legendre-based nodes and polynomial tables.
std::vector<double> gll_points(int p);                  // p+1 GLL points on [0,1]
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);  // on [0,1]
double lagrange_value(const std::vector<double>& nodes, int a, double x);
double lagrange_derivative(const std::vector<double>& nodes, int a, double x);
double bernstein_value(int m, int a, double x);
double bernstein_derivative(int m, int a, double x);

// ---------------------------------------------------------------------------
// Device-side table of small per-problem constants, packed in one buffer.
struct Tables {
  // geometry coefficients: Bernstein gradients at the interpolation points
  int off_geo_dN;      // [nL][(m+1)^2][2]
  int off_chk_dN;      // [nchk][(m+1)^2][2]  det J check sample
  int nchk;
  // constraint rows: Gauss 2p+2 points on an edge
  int nq_edge;
  int off_edge_w;      // [nq]
  int off_edge_b;      // [p+1][nq] GLL Lagrange values
  int off_edge_B;      // [m+1][nq] Bernstein values
  int off_edge_dB;     // [m+1][nq] Bernstein derivatives
  int off_edge_x;      // [nq] the edge rule's Gauss nodes on [0, 1]
  int off_edge_nodes;  // [p+1] GLL nodes
  int off_edge_bw;     // [p+1] barycentric weights 1 / prod_{l != a} (x_a - x_l) of the GLL nodes
  int off_mid_B;       // [m+1] Bernstein values at 1/2
  // loads: Gauss p+2m+2 points
  int nq_load;
  int off_load_w, off_load_b, off_load_dB;
  int off_load_x;      // [nq_load] the load rule's Gauss nodes on [0, 1]
  // MDEIM: GLL points of degree r for each family slot (max 4 families)
  int off_rnodes[4];
  // adjoint chain rule: Bernstein gradients at interpolation points (= geo_dN)
  int total;
};

// cluster index and local coordinates of a cell's thresholds (the clamped
// per-coordinate interval, as in k_geometry; a value outside the box has
// already raised the range flag there)
// GLL Lagrange polynomial n (of p + 1 tabulated nodes, barycentric weights bw)
// at s.
__device__ inline double gll_lagrange(const double* nodes, const double* bw, int p, int n, double s) {
  double v = bw[n];
  for (int l = 0; l <= p; ++l)
    if (l != n) v *= s - nodes[l];
  return v;
}

// Derivatives at s of the m + 1 Bernstein polynomials of degree m (m <= 4):
// dB[k] = m (B_{k-1,m-1}(s) - B_{k,m-1}(s)), the degree m - 1 values by the
// triangular recurrence (no divisions).
__device__ inline void bernstein_deriv_at(int m, double s, double dB[5]) {
  double b[5] = {1.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = 1; j < m; ++j)
    for (int k = j; k >= 0; --k) b[k] = (1.0 - s) * b[k] + (k > 0 ? s * b[k - 1] : 0.0);
  for (int k = 0; k <= m; ++k) dB[k] = m * ((k > 0 ? b[k - 1] : 0.0) - (k < m ? b[k] : 0.0));
}

__device__ inline int mdeim4_cluster(const double* mu, double lo, double hi, int nk, double tau[4], double hstep[4]) {
  const double w = (hi - lo) / nk;
  int k = 0;
  for (int i = 3; i >= 0; --i) {
    const double v = mu[i];
    int ci = (int)floor((v - lo) / w);
    if (ci > nk - 1) ci = nk - 1;
    if (ci < 0) ci = 0;
    const double a = lo + ci * w, b = lo + (ci + 1) * w;
    tau[i] = (v - a) / (b - a);
    hstep[i] = b - a;
    k = k * nk + ci;
  }
  return k;
}

// Lagrange basis value l_a(tau) on the r+1 nodes x, and its derivative
__device__ inline double lag_value(const double* x, int R, int a, double tau) {
  double v = 1.0;
  for (int l = 0; l <= R; ++l)
    if (l != a) v *= (tau - x[l]) / (x[a] - x[l]);
  return v;
}

__device__ inline double lag_deriv(const double* x, int R, int a, double tau) {
  double s = 0.0;
  for (int l = 0; l <= R; ++l) {
    if (l == a) continue;
    double term = 1.0 / (x[a] - x[l]);
    for (int q = 0; q <= R; ++q)
      if (q != a && q != l) term *= (tau - x[q]) / (x[a] - x[q]);
    s += term;
  }
  return s;
}

// A loaded ROM of one family.
struct RomDev {
  int family = -1, p = 0, q = 0, n_k = 0, n_r = 0, r = 0;
  int dim = 1;                      // parameters per cell: 1 (t) or 4 (corner thresholds)
  int ncl = 0;                      // clusters, n_k^dim
  double lo = 0, hi = 0;
  int KC = 0;                       // k-chunks of the contraction (4*KC >= n_r + 1)
  std::vector<double*> ut64;        // per cluster: tiled [NPT][ns][KC][64] FP64
  std::vector<float*> ut32;         // per cluster: tiled [NPT][ns][KC][64] FP32
  std::vector<double*> ucol64;      // per cluster: [NPT][ns][16][4*KC] plain rows (adjoint)
  double* coeff = nullptr;          // [ncl][(r+1)^dim][n_r]
};

// Node of the nested-dissection tree of the coarse problem (same layout on the
// host and the device).  Front = [own dofs | boundary dofs], nf = ns + nb,
// stored row-major at foff; after the partial Gauss-Jordan sweep it holds
// [[F_ss^-1, M^T], [-M, U]] with M = F_bs F_ss^-1 and U the update matrix.
// Fronts of at most this many dofs are swept with the whole front in LDS.
constexpr int ND_LDS_NF = 140;
// Own rows per workgroup of the backward coarse sweep (a multiple of 4).
constexpr int ND_BW_ROWS = 16;

struct NDNodeH {
  long long foff = 0;
  long long cp_off = 0;  // offset of the node's pivot-column panel (blocked levels only)
  int ns = 0, nb = 0, own_off = 0, bnd_off = 0, up_off = 0, beff_off = 0;
  int child[2] = {-1, -1};
  int cmap_off[2] = {-1, -1};
  int parent = -1, level = 0;
};

// One work item of a coarse solve sweep: the node data the item needs, so a
// workgroup starts with a single load.  first = first boundary column
// (forward) or first own row (backward).  Own dofs of a node are the coarse
// dofs [own_off, own_off + ns) (coarse dofs are numbered in tree order).
struct NDItem {
  long long foff;
  int ns, nb, own_off, bnd_off, up_off, first;
  int child_up_off[2], child_nb[2];
  int pull_off;          // forward: the node's pull map (int2 per front position), -1 for a leaf
  int kpart, kparts;     // forward: this item's own-row part and the node's number of parts
  int child_kparts[2];
  int pad[3];
};

// Forward items split the own rows of every node into parts of ND_KPART rows
// (one part per workgroup, 16 rows per wave).  Backward items of levels with
// fewer than ND_SPLIT_NODES nodes take 4 rows each, so the few large fronts of
// the upper tree levels are spread over more workgroups.
constexpr int ND_SPLIT_NODES = 64;
constexpr int ND_KPART = 64;
// The bottom ND_SUB_LEVELS levels of the tree are swept one subtree per
// workgroup (one launch per sweep), when their top level has at least
// ND_SUB_MIN_ROOTS nodes and their fronts fit the per-wave kernels.
constexpr int ND_SUB_LEVELS = 3;
constexpr int ND_SUB_MIN_ROOTS = 256;
constexpr int ND_SUB_MAX_NF = 256;

// The forward sweep of the bottom ND_FUSED_LEVELS levels of the tree can be
// one launch in which a workgroup takes a whole subtree: its factor rows,
// index program and vector entries are all requested at the start and staged
// in LDS, and the levels follow one another with workgroup barriers only.
constexpr int ND_FUSED_LEVELS = 4;
constexpr int ND_FUSED_THREADS = 512;
constexpr int ND_FUSED_LDS_DOUBLES = 19456;   // 152 KiB of LDS per workgroup
constexpr int ND_FUSED_LOADS = 20;            // 16-byte block loads per thread (block <= 2 * 20 * 512 doubles)
constexpr int ND_FUSED_ENT = 4;               // vector entries per thread (<= 4 * 512 per subtree)
constexpr int ND_FUSED_MIN_ROOTS = 64;

// One subtree of the fused sweeps.  Depth d = 0 is the subtree root.
struct FusedSub {
  long long fwd_off;           // its packed M^T block in the fused block buffer (doubles, even)
  int fwd_n;                   // block size (doubles, even)
  int own_off, own_n;          // its own coarse dofs: one contiguous range (tree order)
  int vec_n;                   // doubles of the per-node vector area in LDS
  int node0;                   // first of its nodes in the fused node table
  int stage_node[ND_FUSED_LEVELS + 1];  // node ranges by depth (relative to node0)
  int went[ND_FUSED_LEVELS + 1];        // vector entries by depth (absolute)
  int stage_pairs[ND_FUSED_LEVELS];     // (node, boundary column) pairs by depth
};
// A node of a fused subtree; offsets in doubles: mt in the subtree's block,
// w and up in its LDS vector area, own in its own range; gup = the root's
// global up offset (-1 below the root); pair0 = the node's first (node,
// column) pair among those of its depth.  At most ND_FUSED_STAGE_NODES nodes
// per depth.
constexpr int ND_FUSED_STAGE_NODES = 8;
struct FusedNode {
  int ns, nb, nf, mt, w, up, own, gup, pair0, pad;
};
// Copy program of the fused blocks, per node: the M^T part of its top ns rows.
struct FusedPack {
  long long foff, fdst;
  int ns, nb;
};

struct CoarseLayout {
  // first coarse id of each grid vertex [(ny+1)(nx+1)], horizontal edge [(ny+1) nx]
  // (edge ex of line vy) and vertical edge [ny (nx+1)] (edge between lines ey and
  // ey+1 at vx), -1 on a clamped side; numbered grid line by grid line
  std::vector<int> vert_first, hedge_first, vedge_first;
  // unique entries of S_C: entry e sums contributions [cstart[e], cstart[e+1]) into dest[e]
  std::vector<long long> dest;        // position in the front storage
  std::vector<int> cstart;
  std::vector<int> contrib;           // index into ScLoc (cell*nCp + packed)
  // nested dissection
  std::vector<NDNodeH> nd_nodes;
  std::vector<int> nd_own, nd_bnd, nd_cmap;  // own/boundary coarse ids per node (tree-order numbering)
  // pull maps of the forward sweep: for each front position of a node with
  // children, the index of that position in child 0's and child 1's boundary
  // (-1 where the child does not touch it); the inverse of nd_cmap
  std::vector<int> nd_pull;
  std::vector<std::vector<int>> nd_levels;   // node ids per depth (0 = root)
  long long nd_front_total = 0;
  int nd_up_total = 0, nd_beff_total = 0, nd_nfmax = 0, nd_nsmax = 0;
  long long nd_cp_total = 0;  // panel scratch of the largest blocked level
  // per-level work lists of the solve sweeps: (node, first row) items
  std::vector<NDItem> fw_items, bw_items;
  std::vector<int2> fw_src, sub_fw_src;     // per forward item, 128 gather sources (see push_fw)
  std::vector<int> lvl_nodes;
  std::vector<int> fw_off, bw_off, lvl_off;
  std::vector<int> lvl_nfmax, lvl_nsmax;  // largest front and own-block size per level
  std::vector<int> lvl_bw_rows;           // own rows per backward item on each level (4 or ND_BW_ROWS)
  std::vector<int> lvl_fw_rows;           // largest own-row part of a forward item on each level
  std::vector<int> lvl_child_kparts;      // largest number of row parts of a child on each level
  // bottom levels [sub_level, L) swept one subtree per workgroup (sub_level = L: none):
  // items of subtree t, stage s in [off[t (nst + 1) + s], off[t (nst + 1) + s + 1])
  int sub_level = 0, sub_nst = 0, sub_count = 0;
  int sub_fw_rows = 0, sub_child_kparts = 0, sub_nfmax = 0;
  std::vector<NDItem> sub_fw_items, sub_bw_items;
  std::vector<int> sub_fw_off, sub_bw_off;
  // fused bottom-level sweeps (used when `fused`, levels [fused_level, L))
  bool fused = false;
  int fused_level = 0;
  std::vector<FusedSub> f_subs;
  std::vector<FusedNode> f_nodes;
  std::vector<short4> f_went;   // {W index, child-0 up index, child-1 up index, own index} (-1: none)
  std::vector<FusedPack> f_pack;
  long long f_blk_total = 0;
};


struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::map<int, RomDev> roms;

  // problem
  bool have_problem = false, assembled = false, setup_done = false, solved = false;
  lbddc_precision asm_prec = LBDDC_FP64, setup_prec = LBDDC_FP64;
  int nx = 0, ny = 0, p = 0, q = 0, m = 0, nrhs = 1;
  double E = 1, nu = 0.3, rho = 0;
  bool moments = true;
  uint32_t clamped = LBDDC_SIDE_LEFT;  // clamped sides (LBDDC_SIDE_* set)
  int load_edge = 1;                   // loaded side as a cell edge: 0 left, 1 right, 2 bottom, 3 top
  int n_side = 0;                      // cell edges along the loaded side
  int ncell = 0, nB = 0, ndof = 0, nI = 0, nU = 0, nE = 0, nC = 0, nce = 0, nL = 0, ns = 0;
  int nN = 0, npair = 0, NPT = 0, nIn = 0, Gx = 0, Gy = 0, netx = 0, nety = 0;
  long long n_i = 0;
  int NU = 0, NI = 0, NC = 0, Nfree = 0;
  int KC = 0;                // contraction k-chunks for this problem (max over families)
  std::vector<int> fam_host; std::vector<double> t_host;
  std::vector<int> fam_slot; // family id -> 0..nfam-1
  std::vector<int> fam_ids;

  // host topology
  std::vector<int> perm_nat;   // permuted node -> natural node index
  std::vector<int> RU, RC;     // [ncell][nU], [ncell][nC]
  CoarseLayout co;
  Tables tab;

  // device buffers -------------------------------------------------------
  double* d_tab = nullptr;
  double* d_ctrl = nullptr;    // [nety][netx][2]
  int* d_family = nullptr;
  double* d_t = nullptr;
  double* d_trac = nullptr;    // [nrhs][n_side][2]
  double* d_ctrl_bak = nullptr;  // the previous control net, t and mu while new ones are validated
  double* d_t_bak = nullptr;
  double* d_mu = nullptr;      // [ncell][4] corner thresholds (cells of dim-4 families)
  double* d_mu_bak = nullptr;
  bool any_dim4 = false;       // some family of the problem has four parameters per cell
  std::vector<int> tile_fam_first, tile_fam_n;  // each family's range of the contraction's 128-cell tiles
  int* d_perm = nullptr;       // [nN]
  int* d_RU = nullptr;         // [ncell][nU]
  int* d_RC = nullptr;         // [ncell][nC]
  int* d_uown_ptr = nullptr;   // [NU+1]
  int* d_uown = nullptr;       // owner slot ids cell*nU + slot
  int* d_cown_ptr = nullptr;   // [NC+1]
  int* d_cown = nullptr;
  // the same owner lists at a fixed width of 4 (-1: none; a skeleton or coarse
  // dof belongs to at most the 4 cells around a vertex), for one-load gathers
  int4* d_uown4 = nullptr;     // [NU]
  int4* d_cown4 = nullptr;     // [NC]
  int* d_skel_node = nullptr;  // [NU/2] node lattice index of each skeleton node
  int* d_net_ptr = nullptr;    // [netx*nety+1]
  int* d_net_own = nullptr;    // cell*(m+1)^2 + local control point
  int* d_cstart = nullptr; int* d_contrib = nullptr; long long* d_dest = nullptr;
  NDNodeH* d_nd_nodes = nullptr;
  int *d_nd_bnd = nullptr, *d_nd_cmap = nullptr;
  int2 *d_fw_src = nullptr, *d_sub_fw_src = nullptr;
  NDItem *d_fw_items = nullptr, *d_bw_items = nullptr;
  NDItem *d_sub_fw_items = nullptr, *d_sub_bw_items = nullptr;
  FusedSub* d_f_subs = nullptr;
  FusedNode* d_f_nodes = nullptr;
  short4* d_f_went = nullptr;
  FusedPack* d_f_pack = nullptr;
  double* d_f_blk = nullptr;    // packed factor rows of the fused subtrees
  int *d_sub_fw_off = nullptr, *d_sub_bw_off = nullptr;
  int* d_lvl_nodes = nullptr;
  int* d_flags = nullptr;      // device error flags [8]
  int* h_flags = nullptr;      // pinned host mirror

  // assembly
  double* d_theta = nullptr;   // [ncell][ns][4]
  double* d_itil = nullptr;    // [ncell][4*KC]
  float* d_theta32 = nullptr;
  float* d_itil32 = nullptr;
  int* d_cluster = nullptr;    // [ncell] group id
  int* d_sorted = nullptr;     // [ncell] cells sorted by group
  // theta of the cells of each contraction tile, step-major: [tile][ns][128][4]
  // (one 16-cell block of one step is 16 consecutive entries); the gradient
  // reuses the FP64 buffer for its 16-cell tiles ([tile][ns][16][4])
  double* d_theta_t = nullptr;
  float* d_theta_t32 = nullptr;
  int* d_tiles = nullptr;      // [ntiles][4]: group, start, count, -
  int ntiles = 0;
  double* d_K = nullptr;       // [ncell][npair][4]
  float* d_K32 = nullptr;       // FP32 contraction ([ncell][npair][4]), valid while k32_valid
  bool k32_valid = false;
  double* d_load = nullptr;    // [nrhs][ncell][nU]
  double* d_cons = nullptr;    // [ncell][4][nce][p+1][2] edge constraint rows
  std::vector<int> group_family, group_cluster;

  // setup
  double* d_S = nullptr;       // [ncell][nU(nU+1)/2]
  double* d_W = nullptr;       // [ncell][schur_w_count(p)] interior elimination multipliers
  double* d_diagK = nullptr;   // [ncell][nU]
  double* d_Ktot = nullptr;    // [NU]
  void* d_P = nullptr;         // [ncell][nE(nE+1)/2] D-scaled fine operator (T)
  void* d_Psi = nullptr;       // [ncell][nC][nU] D-scaled coarse basis (T), column by column
  double* d_D = nullptr;       // [ncell][nU]
  double* d_ScLoc = nullptr;   // [ncell][nC(nC+1)/2]
  double* d_coarse = nullptr;  // nested-dissection fronts
  double* d_up = nullptr;      // per node up-vectors of the forward sweep
  double* d_beff = nullptr;    // per node effective right-hand sides
  double* d_gjC = nullptr;     // pivot-column panels of the blocked front sweep

  // solve
  double* d_f = nullptr;       // [nrhs][NU]
  double* d_x = nullptr;       // [nrhs][NU]
  double *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_q = nullptr;
  double* d_partU = nullptr;   // [ncell][nU]
  double* d_partC = nullptr;   // [ncell][nC]
  double *d_zc = nullptr, *d_tc = nullptr, *d_xc = nullptr;  // coarse vectors [NC]
  double* d_red = nullptr;     // reduction partials [kRedSlots][kMaxBlocks]
  double* d_scal = nullptr;    // scalars, scal_stride() per load case of a block
  double* d_hred = nullptr;    // h_red as a device address (kernels write the r.r partials there)
  double* h_scal = nullptr;    // pinned
  double* d_vred = nullptr;    // interface-vector partials: p.q, r.z, r.r [3][NU / 256 + 16]
  double* h_red = nullptr;     // pinned, coherent: the r.r partials and breakdown flag of the last update
  // The iteration vectors r, z, p, q (NU), the cell partials, the coarse
  // vectors zc, xc (NC), the sweep vectors up and beff, the scalars, the
  // interface partials and the pinned poll buffer hold nblk load cases, one
  // after another.
  int nblk = 1;
  size_t scal_stride() const { return (size_t)(32 + NU / 1024 + 16); }
  size_t vred_stride() const { return (size_t)3 * (NU / 256 + 16); }
  double* d_u = nullptr;       // [nrhs][Gy][Gx][2]
  std::vector<lbddc_solve_info> info;

  // gradient
  double* d_H = nullptr;       // [ncell][4*KC]
  double* d_G = nullptr;       // [ncell][ns][4]
  double* d_gcell = nullptr;   // [ncell][(m+1)^2][2]
  double* d_edge_br = nullptr; // [ncell * 4][16] sorted breaks of each edge's material part (Table 1 cells)
  int* d_edge_nm = nullptr;    // [ncell * 4][2] break count and material-interval mask (-1: whole edge)
  double* d_gt = nullptr;      // [nrhs][ncell]
  double* d_gmu = nullptr;     // [nrhs][ncell][4]
  double* d_gX = nullptr;      // [nrhs][nety*netx*2]
  double* d_J = nullptr;       // [nrhs]
  int* d_adj_tiles = nullptr;  // 16-cell tiles of the adjoint contraction
  void* d_adj_ptrs = nullptr;  // per-group tile pointers (A and transposed layouts)
  std::vector<int> group_counts;
  // Generation of the geometry (t, family): bumped by set_geometry_device.
  // The assembly's group sort, tile table and per-group pointers depend on it
  // only, so an assembly with an unchanged generation into the same buffers
  // reuses them and skips the host round trip of the sort.
  unsigned long long geom_gen = 1;
  struct GroupCache {
    unsigned long long gen = 0;
    bool fp32 = false;
    const void* tiles = nullptr;
    int ntiles = 0;
    std::vector<int> fam_first, fam_n;
  } grp;
  double* d_ucell = nullptr;   // [ncell][ndof] local displacement (permuted)

  double phase_ms[15] = {0};
  static constexpr int kNumEv = 9;
  hipEvent_t ev[kNumEv] = {};
  // a second stream (default priority) for the edge rows and loads of
  // four-parameter lattices, which run beside the geometry pass and the
  // contraction; fork and join events without timing
  hipStream_t side = nullptr;
  hipEvent_t side_fork = nullptr, side_join = nullptr;
  // events of the timed PCG phases, a ring of kRing iterations read back at the
  // end of the solve (no host wait inside the loop): per slot [0, 1] operator,
  // [2, 3] preconditioner local kernel, [4, 5, 6] coarse solve start, between
  // the sweeps, end
  static constexpr int kRing = 8, kRingEv = 7;
  hipEvent_t pev[kRing][kRingEv] = {};
  int timing = LBDDC_TIME_ALL;  // PCG phases timed (LBDDC_TIME_* mask)
  size_t dev_bytes = 0;
  std::vector<void*> allocs;   // everything allocated for the problem
};

// allocation helpers (api.cpp)
bool dalloc(Ctx* c, void** p, size_t bytes);
template <class T> bool dalloc_t(Ctx* c, T** p, size_t n) { return dalloc(c, (void**)p, n * sizeof(T)); }

// topology (topology.cpp)
bool build_topology(Ctx* c);
bool build_nested_dissection(Ctx* c, const std::vector<int>& ent_g1, const std::vector<int>& ent_g2);
void build_fused_sweeps(Ctx* c);
void build_tables(Ctx* c, std::vector<double>& tab);

// ---------------------------------------------------------------------------
// Kernel launchers.  All enqueue on c->stream and return hipGetLastError().
hipError_t launch_geometry(Ctx* c);          // theta, det check, MDEIM eval (A1, A2)
// MDEIM evaluation of a four-parameter family over its tiles [first, first + n)
// of the cluster-sorted cell order (after the group sort of the contraction)
hipError_t launch_mdeim4(Ctx* c, int slot, const int* d_tiles, int first, int n);
hipError_t launch_constraints_loads(Ctx* c, hipStream_t st); // edge constraint rows and loads
hipError_t launch_assembly(Ctx* c, bool fp32, hipEvent_t e0, hipEvent_t e1);  // A3
hipError_t noalloc_scratch_init(int device);                          // address of the static scratch (device current)
lbddc_status assemble_fp32_noalloc(Ctx* c, float* d_K);               // A3, FP32, caller's output, static scratch
hipError_t launch_theta_tile16(Ctx* c, const int4* tiles, int ntiles, double* out);  // A11 (theta in tile order)
hipError_t launch_schur(Ctx* c);             // A4
hipError_t launch_weights(Ctx* c);           // A7 (gather of stiffness diagonals)
hipError_t launch_precond(Ctx* c, bool fp32); // A5, A6, A7
hipError_t launch_coarse_assemble(Ctx* c);   // A8 assembly of S_C blocks
hipError_t prepare_fused_sweeps(Ctx* c);     // LDS limit of the fused bottom-level sweeps
hipError_t launch_coarse_factor(Ctx* c);     // A8 nested-dissection FP64 factorization (and the fused blocks)
// The load cases of one coarse sweep launch, all served by every workgroup:
// load case y has its right-hand side and solution y * v doubles after the first,
// its up vectors y * up and its effective right-hand sides y * beff doubles
// further; cases whose bit in mask is clear are skipped.
struct SweepVecs {
  long long v, up, beff;
  unsigned mask;
  int nr;  // load cases 0 .. nr - 1 (those with their bit in mask are solved)
};
// A8 solve of nr load cases at once (right-hand sides rhs + k NC, solutions
// x + k NC; the cases with a clear bit in mask are left untouched)
hipError_t launch_coarse_solve(Ctx* c, const double* rhs, double* x, hipEvent_t mid = nullptr, int nr = 1,
                               unsigned mask = 1u);
hipError_t pcg_solve(Ctx* c, int rhs, double rtol, int max_iter, lbddc_solve_info* info, bool fp32,
                     double* t_op, double* t_pre, double* t_coarse, double* t_cfwd, double* t_cbwd,
                     int* n_apply);  // A9
hipError_t pcg_solve_block(Ctx* c, int r0, int nr, double rtol, int max_iter, lbddc_solve_info* info, bool fp32,
                           double* t_op, double* t_pre, double* t_coarse, double* t_cfwd, double* t_cbwd,
                           int* n_apply, int* n_op);  // A9, nr <= kBlockRhs load cases at once
hipError_t pcg_true_residual(Ctx* c, int rhs, double* out);
hipError_t gather_rhs(Ctx* c, int rhs);
hipError_t launch_recover(Ctx* c, int rhs);  // A10
hipError_t launch_gradient(Ctx* c, int rhs); // A11
hipError_t launch_export(Ctx* c, int which, int first, int count, double* d_out);

}  // namespace lbddc

struct lbddc_ctx {
  lbddc::Ctx c;
};
