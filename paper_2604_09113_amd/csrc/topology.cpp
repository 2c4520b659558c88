// Host-side index maps of the lattice (integer topology only) and the small
// polynomial tables the kernels read.
//
// Dof classification (Sec. 3.1): nodes on the clamped sides are Dirichlet,
// the (p-1)^2 nodes strictly inside a cell are interior, every other node is a
// skeleton node (this reading reproduces the dof counts printed for the
// weak-scaling study).  Coarse dofs (Sec. 3.3.1): two values per non-Dirichlet
// grid vertex, two averages and (optionally) one moment per non-Dirichlet edge.
//
// Coarse numbering by grid lines: line j holds the vertices and horizontal
// edges of y = j followed by the vertical edges between y = j and y = j + 1
// (vertices and edges on clamped sides carry no coarse dof).
// The elimination order of the coarse problem is a nested dissection of the
// cell grid (nd.cpp); this numbering only names the coarse dofs.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace lbddc {

static int skel_node_local(int p, int node, int& a, int& b) {
  // canonical skeleton node slots: BL, BR, TL, TR, left, right, bottom, top
  if (node < 4) {
    a = (node & 1) ? p : 0;
    b = (node & 2) ? p : 0;
    return 0;
  }
  int e = (node - 4) / (p - 1), k = (node - 4) % (p - 1) + 1;
  if (e == 0) { a = 0; b = k; }
  else if (e == 1) { a = p; b = k; }
  else if (e == 2) { a = k; b = 0; }
  else { a = k; b = p; }
  return 0;
}

bool build_topology(Ctx* c) {
  const int p = c->p, nx = c->nx, ny = c->ny, nU = c->nU, nC = c->nC, nce = c->nce;
  // permuted node order: interior nodes, then skeleton slots
  c->perm_nat.assign(c->nN, 0);
  int n = 0;
  for (int b = 1; b < p; ++b)
    for (int a = 1; a < p; ++a) c->perm_nat[n++] = a + (p + 1) * b;
  for (int s = 0; s < 4 * p; ++s) {
    int a, b;
    skel_node_local(p, s, a, b);
    c->perm_nat[n++] = a + (p + 1) * b;
  }
  const bool cl_l = c->clamped & LBDDC_SIDE_LEFT, cl_r = c->clamped & LBDDC_SIDE_RIGHT;
  const bool cl_b = c->clamped & LBDDC_SIDE_BOTTOM, cl_t = c->clamped & LBDDC_SIDE_TOP;
  // global skeleton numbering (every lattice node on a grid line except the
  // nodes of the clamped sides), band by band: grid line y = iy p with its nodes in
  // increasing x, then the interior nodes of the vertical edges between lines
  // iy and iy + 1, edge by edge in increasing x and each edge in increasing y.
  // The nodes of every cell edge are then consecutive, as are the slots the
  // two cells sharing the edge give them, so the sums over a dof's cells and
  // the per-cell gathers of interface vectors read contiguous runs.
  const int Gx = c->Gx, Gy = c->Gy;
  auto node_dir = [&](int gx, int gy) {
    return (cl_l && gx == 0) || (cl_r && gx == Gx - 1) || (cl_b && gy == 0) || (cl_t && gy == Gy - 1);
  };
  std::vector<int> sk((size_t)Gx * Gy, -1);
  int nsk = 0;
  std::vector<int> sk_node;
  auto add = [&](int gx, int gy) {
    if (node_dir(gx, gy)) return;
    sk[(size_t)gy * Gx + gx] = nsk++;
    sk_node.push_back(gy * Gx + gx);
  };
  for (int iy = 0; iy <= ny; ++iy) {
    for (int gx = 0; gx < Gx; ++gx) add(gx, p * iy);
    if (iy < ny)
      for (int vx = 0; vx <= nx; ++vx)
        for (int k = 1; k < p; ++k) add(p * vx, p * iy + k);
  }
  c->NU = 2 * nsk;
  c->RU.assign((size_t)c->ncell * nU, -1);
  for (int cell = 0; cell < c->ncell; ++cell) {
    int ix = cell % nx, iy = cell / nx;
    for (int s = 0; s < 4 * p; ++s) {
      int a, b;
      skel_node_local(p, s, a, b);
      int id = sk[(size_t)(p * iy + b) * Gx + p * ix + a];
      for (int comp = 0; comp < 2; ++comp)
        c->RU[(size_t)cell * nU + 2 * s + comp] = id >= 0 ? 2 * id + comp : -1;
    }
  }
  // coarse numbering by grid lines: line j holds the vertices and horizontal
  // edges of y = j, then the vertical edges between y = j and y = j + 1
  CoarseLayout& co = c->co;
  const auto on_x = [&](int vx) { return (cl_l && vx == 0) || (cl_r && vx == nx); };
  const auto on_y = [&](int vy) { return (cl_b && vy == 0) || (cl_t && vy == ny); };
  co.vert_first.assign((size_t)(ny + 1) * (nx + 1), -1);
  co.hedge_first.assign((size_t)(ny + 1) * nx, -1);
  co.vedge_first.assign((size_t)ny * (nx + 1), -1);
  int off = 0;
  for (int vy = 0; vy <= ny; ++vy) {
    for (int vx = 0; vx <= nx; ++vx)
      if (!on_x(vx) && !on_y(vy)) { co.vert_first[(size_t)vy * (nx + 1) + vx] = off; off += 2; }
    for (int ex = 0; ex < nx; ++ex)
      if (!on_y(vy)) { co.hedge_first[(size_t)vy * nx + ex] = off; off += nce; }
    if (vy < ny)
      for (int vx = 0; vx <= nx; ++vx)
        if (!on_x(vx)) { co.vedge_first[(size_t)vy * (nx + 1) + vx] = off; off += nce; }
  }
  c->NC = off;
  auto vert = [&](int vx, int vy) { return co.vert_first[(size_t)vy * (nx + 1) + vx]; };
  auto hedge = [&](int ex, int vy) { return co.hedge_first[(size_t)vy * nx + ex]; };
  auto vedge = [&](int vx, int ey) { return co.vedge_first[(size_t)ey * (nx + 1) + vx]; };
  c->RC.assign((size_t)c->ncell * nC, -1);
  for (int cell = 0; cell < c->ncell; ++cell) {
    int ix = cell % nx, iy = cell / nx;
    int* r = &c->RC[(size_t)cell * nC];
    int v[4] = {vert(ix, iy), vert(ix + 1, iy), vert(ix, iy + 1), vert(ix + 1, iy + 1)};
    for (int k = 0; k < 4; ++k)
      for (int comp = 0; comp < 2; ++comp) r[2 * k + comp] = v[k] >= 0 ? v[k] + comp : -1;
    int e[4] = {vedge(ix, iy), vedge(ix + 1, iy), hedge(ix, iy), hedge(ix, iy + 1)};
    for (int k = 0; k < 4; ++k)
      for (int t2 = 0; t2 < nce; ++t2) r[8 + nce * k + t2] = e[k] >= 0 ? e[k] + t2 : -1;
  }
  // owner lists (in increasing cell order: fixed summation order)
  auto owners = [](const std::vector<int>& R, int N, std::vector<int>& ptr, std::vector<int>& own) {
    ptr.assign(N + 1, 0);
    for (size_t i = 0; i < R.size(); ++i)
      if (R[i] >= 0) ptr[R[i] + 1]++;
    for (int g = 0; g < N; ++g) ptr[g + 1] += ptr[g];
    own.assign(ptr[N], 0);
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < R.size(); ++i)
      if (R[i] >= 0) own[fill[R[i]]++] = (int)i;
  };
  std::vector<int> uptr, uown, cptr, cown;
  owners(c->RU, c->NU, uptr, uown);
  owners(c->RC, c->NC, cptr, cown);

  // unique entries of S_C with their contributions in increasing cell order
  const int nCp = nC * (nC + 1) / 2;
  std::vector<int> ent_g1, ent_g2;
  co.cstart.assign(1, 0);
  co.contrib.clear();
  std::vector<std::pair<long long, int>> row;
  for (int g1 = 0; g1 < c->NC; ++g1) {
    row.clear();
    for (int o = cptr[g1]; o < cptr[g1 + 1]; ++o) {
      int slot = cown[o];
      int cell = slot / nC, l1 = slot % nC;
      for (int l2 = 0; l2 < nC; ++l2) {
        int g2 = c->RC[(size_t)cell * nC + l2];
        if (g2 < 0) continue;
        int hi = std::max(l1, l2), lo = std::min(l1, l2);
        row.push_back({(long long)g2 * c->ncell + cell, cell * nCp + hi * (hi + 1) / 2 + lo});
      }
    }
    std::sort(row.begin(), row.end());
    size_t i = 0;
    while (i < row.size()) {
      int g2 = (int)(row[i].first / c->ncell);
      size_t k = i;
      while (k < row.size() && (int)(row[k].first / c->ncell) == g2) {
        co.contrib.push_back(row[k].second);
        ++k;
      }
      co.cstart.push_back((int)co.contrib.size());
      ent_g1.push_back(g1);
      ent_g2.push_back(g2);
      i = k;
    }
  }
  if (!build_nested_dissection(c, ent_g1, ent_g2)) return false;
  // renumber the coarse dofs in tree order (node by node, own dofs in the
  // order of the node's own list), so a node's own dofs are a contiguous range
  {
    std::vector<int> newid(c->NC, -1);
    for (size_t i = 0; i < co.nd_own.size(); ++i) newid[co.nd_own[i]] = (int)i;
    for (int& r : c->RC)
      if (r >= 0) r = newid[r];
    for (int& g : co.nd_bnd) g = newid[g];
    for (size_t i = 0; i < co.nd_own.size(); ++i) co.nd_own[i] = (int)i;
    owners(c->RC, c->NC, cptr, cown);
  }
  // solve work lists: forward items = 64-column chunks of the boundary (at
  // least one per node) x 64-row parts of the own rows, backward items = runs
  // of own rows.  The forward result of a node is stored as kparts partial
  // vectors of nb entries (kp-major), which the parent adds in a fixed order.
  const int L = (int)co.nd_levels.size();
  std::vector<int> kparts(co.nd_nodes.size(), 1);
  for (size_t n = 0; n < co.nd_nodes.size(); ++n)
    kparts[n] = std::max(1, (co.nd_nodes[n].ns + ND_KPART - 1) / ND_KPART);
  // pull maps: inverse of the child maps, two entries per front position
  std::vector<int> pull_off(co.nd_nodes.size(), -1);
  co.nd_pull.clear();
  for (size_t n = 0; n < co.nd_nodes.size(); ++n) {
    const NDNodeH& d = co.nd_nodes[n];
    if (d.child[0] < 0 && d.child[1] < 0) continue;
    const size_t base = co.nd_pull.size();
    pull_off[n] = (int)(base / 2);
    co.nd_pull.resize(base + 2 * (size_t)(d.ns + d.nb), -1);
    for (int s = 0; s < 2; ++s) {
      const int ch = d.child[s];
      if (ch < 0) continue;
      for (int i = 0; i < co.nd_nodes[ch].nb; ++i) {
        const int pos = co.nd_cmap[d.cmap_off[s] + i];
        if (pos < 0 || pos >= d.ns + d.nb || co.nd_pull[base + 2 * pos + s] != -1) {
          c->err = "internal: a child map that is not one-to-one";
          return false;
        }
        co.nd_pull[base + 2 * pos + s] = i;
      }
    }
  }
  // one spare position, so the maps are never empty: the forward sweep reads
  // entry 0 for leaves and for positions it does not need
  co.nd_pull.push_back(-1);
  co.nd_pull.push_back(-1);
  {
    int uoff = 0;
    for (size_t n = 0; n < co.nd_nodes.size(); ++n) {
      co.nd_nodes[n].up_off = uoff;
      uoff += kparts[n] * co.nd_nodes[n].nb;
    }
    co.nd_up_total = uoff;
  }
  auto make_item = [&](int n) {
    const NDNodeH& d = co.nd_nodes[n];
    NDItem it{};
    it.foff = d.foff;
    it.ns = d.ns;
    it.nb = d.nb;
    it.own_off = d.own_off;
    it.bnd_off = d.bnd_off;
    it.up_off = d.up_off;
    it.kparts = kparts[n];
    for (int s = 0; s < 2; ++s) {
      const int ch = d.child[s];
      it.child_up_off[s] = ch >= 0 ? co.nd_nodes[ch].up_off : 0;
      it.child_nb[s] = ch >= 0 ? co.nd_nodes[ch].nb : 0;
      it.child_kparts[s] = ch >= 0 ? kparts[ch] : 0;
    }
    it.pull_off = pull_off[n];
    return it;
  };
  // A forward item reads the children's up vectors at 128 front positions:
  // its own rows kb + t (t < 64) and, for part 0, its boundary columns
  // first + t - 64 (t >= 64).  src holds, per item and position, the index in
  // `up` of part 0 of each child's entry there (-1: no entry), so that the
  // item's gathers wait for one load instead of two.
  auto push_fw = [&](int n, std::vector<NDItem>& out, std::vector<int2>& src) {
    NDItem it = make_item(n);
    const NDNodeH& d = co.nd_nodes[n];
    for (int kp = 0; kp < kparts[n]; ++kp)
      for (int r = 0; r < std::max(1, d.nb); r += 64) {
        it.first = r;
        it.kpart = kp;
        out.push_back(it);
        const int kb = kp * ND_KPART, ke = std::min(d.ns, kb + ND_KPART);
        for (int t = 0; t < 128; ++t) {
          int j = -1;
          if (t < 64 && kb + t < ke) j = kb + t;
          if (t >= 64 && kp == 0 && r + t - 64 < d.nb) j = d.ns + r + t - 64;
          int2 e = make_int2(-1, -1);
          if (j >= 0 && pull_off[n] >= 0) {
            const int s0 = co.nd_pull[2 * ((size_t)pull_off[n] + j)], s1 = co.nd_pull[2 * ((size_t)pull_off[n] + j) + 1];
            if (s0 >= 0) e.x = it.child_up_off[0] + s0;
            if (s1 >= 0) e.y = it.child_up_off[1] + s1;
          }
          src.push_back(e);
        }
      }
  };
  auto push_bw = [&](int n, int rows, std::vector<NDItem>& out) {
    NDItem it = make_item(n);
    it.kpart = 0;
    for (int r = 0; r < std::max(1, co.nd_nodes[n].ns); r += rows) {
      it.first = r;
      out.push_back(it);
    }
  };
  co.fw_items.clear(); co.bw_items.clear(); co.lvl_nodes.clear(); co.fw_src.clear(); co.sub_fw_src.clear();
  co.fw_off.assign(1, 0); co.bw_off.assign(1, 0); co.lvl_off.assign(1, 0);
  co.lvl_nfmax.assign(L, 0);
  co.lvl_nsmax.assign(L, 0);
  co.lvl_bw_rows.assign(L, ND_BW_ROWS);
  co.lvl_fw_rows.assign(L, 0);
  co.lvl_child_kparts.assign(L, 0);
  for (int l = 0; l < L; ++l) {
    const bool split = (int)co.nd_levels[l].size() < ND_SPLIT_NODES;
    co.lvl_bw_rows[l] = split ? 4 : ND_BW_ROWS;
    for (int n : co.nd_levels[l]) {
      const NDNodeH& d = co.nd_nodes[n];
      co.lvl_nfmax[l] = std::max(co.lvl_nfmax[l], d.ns + d.nb);
      co.lvl_nsmax[l] = std::max(co.lvl_nsmax[l], d.ns);
      co.lvl_fw_rows[l] = std::max(co.lvl_fw_rows[l], std::min(d.ns, ND_KPART));
      for (int s = 0; s < 2; ++s)
        if (d.child[s] >= 0) co.lvl_child_kparts[l] = std::max(co.lvl_child_kparts[l], kparts[d.child[s]]);
      push_fw(n, co.fw_items, co.fw_src);
      push_bw(n, co.lvl_bw_rows[l], co.bw_items);
      co.lvl_nodes.push_back(n);
    }
    co.fw_off.push_back((int)co.fw_items.size());
    co.bw_off.push_back((int)co.bw_items.size());
    co.lvl_off.push_back((int)co.lvl_nodes.size());
  }
  // subtree sweeps of the bottom levels
  co.sub_level = L;
  co.sub_nst = 0;
  co.sub_count = 0;
  co.sub_fw_items.clear(); co.sub_bw_items.clear(); co.sub_fw_off.clear(); co.sub_bw_off.clear();
  {
    const int ls = L - ND_SUB_LEVELS;
    bool use = ls >= 1 && (int)co.nd_levels[ls].size() >= ND_SUB_MIN_ROOTS;
    for (int l = std::max(ls, 0); use && l < L; ++l) use = co.lvl_nfmax[l] <= ND_SUB_MAX_NF;
    if (use) {
      co.sub_level = ls;
      co.sub_nst = L - ls;
      co.sub_count = (int)co.nd_levels[ls].size();
      co.sub_fw_rows = co.sub_child_kparts = co.sub_nfmax = 0;
      for (int l = ls; l < L; ++l) {
        co.sub_fw_rows = std::max(co.sub_fw_rows, co.lvl_fw_rows[l]);
        co.sub_child_kparts = std::max(co.sub_child_kparts, co.lvl_child_kparts[l]);
        co.sub_nfmax = std::max(co.sub_nfmax, co.lvl_nfmax[l]);
      }
      for (int root : co.nd_levels[ls]) {
        // nodes of the subtree by level
        std::vector<std::vector<int>> by(co.sub_nst);
        std::vector<int> stack{root};
        while (!stack.empty()) {
          const int n = stack.back();
          stack.pop_back();
          by[co.nd_nodes[n].level - ls].push_back(n);
          for (int s2 = 1; s2 >= 0; --s2)
            if (co.nd_nodes[n].child[s2] >= 0) stack.push_back(co.nd_nodes[n].child[s2]);
        }
        for (auto& v : by) std::sort(v.begin(), v.end());
        for (int st = 0; st < co.sub_nst; ++st) {
          co.sub_fw_off.push_back((int)co.sub_fw_items.size());
          for (int n : by[co.sub_nst - 1 - st]) push_fw(n, co.sub_fw_items, co.sub_fw_src);
        }
        co.sub_fw_off.push_back((int)co.sub_fw_items.size());
        for (int st = 0; st < co.sub_nst; ++st) {
          co.sub_bw_off.push_back((int)co.sub_bw_items.size());
          for (int n : by[st]) push_bw(n, ND_BW_ROWS, co.sub_bw_items);
        }
        co.sub_bw_off.push_back((int)co.sub_bw_items.size());
      }
    }
  }

  // the fused bottom-level sweeps, when every subtree fits
  build_fused_sweeps(c);

  // fixed-width owner tables (taken after the coarse renumbering)
  auto owners4 = [&](const std::vector<int>& ptr, const std::vector<int>& own, int N, std::vector<int4>& out) {
    out.assign(N, make_int4(-1, -1, -1, -1));
    for (int g = 0; g < N; ++g) {
      const int n = ptr[g + 1] - ptr[g];
      if (n > 4) return false;
      int v[4] = {-1, -1, -1, -1};
      for (int k = 0; k < n; ++k) v[k] = own[ptr[g] + k];
      out[g] = make_int4(v[0], v[1], v[2], v[3]);
    }
    return true;
  };
  std::vector<int4> uown4, cown4;
  if (!owners4(uptr, uown, c->NU, uown4) || !owners4(cptr, cown, c->NC, cown4)) {
    c->err = "internal: a dof with more than 4 owning cells";
    return false;
  }

  // net owners for the gradient gather
  const int m = c->m, np1 = (m + 1) * (m + 1);
  std::vector<int> nptr((size_t)c->netx * c->nety + 1, 0), nown;
  for (int cell = 0; cell < c->ncell; ++cell) {
    int ix = cell % nx, iy = cell / nx;
    for (int b = 0; b <= m; ++b)
      for (int a = 0; a <= m; ++a) nptr[(size_t)(m * iy + b) * c->netx + m * ix + a + 1]++;
  }
  for (size_t g = 0; g + 1 < nptr.size(); ++g) nptr[g + 1] += nptr[g];
  nown.assign(nptr.back(), 0);
  {
    std::vector<int> fill(nptr.begin(), nptr.end() - 1);
    for (int cell = 0; cell < c->ncell; ++cell) {
      int ix = cell % nx, iy = cell / nx;
      for (int b = 0; b <= m; ++b)
        for (int a = 0; a <= m; ++a) {
          size_t g = (size_t)(m * iy + b) * c->netx + m * ix + a;
          nown[fill[g]++] = cell * np1 + b * (m + 1) + a;
        }
    }
  }

  // ---- upload ------------------------------------------------------------------
  auto up = [&](auto** dptr, const auto& v) -> bool {
    using T = typename std::remove_reference<decltype(v)>::type::value_type;
    size_t nbytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (!dalloc(c, (void**)dptr, nbytes)) return false;
    if (!v.empty() && hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
      c->err = "hipMemcpy failed";
      return false;
    }
    return true;
  };
  return up(&c->d_perm, c->perm_nat) && up(&c->d_RU, c->RU) &&
         up(&c->d_RC, c->RC) && up(&c->d_uown_ptr, uptr) && up(&c->d_uown, uown) && up(&c->d_cown_ptr, cptr) &&
         up(&c->d_cown, cown) && up(&c->d_uown4, uown4) && up(&c->d_cown4, cown4) && up(&c->d_skel_node, sk_node) && up(&c->d_net_ptr, nptr) &&
         up(&c->d_net_own, nown) && up(&c->d_cstart, co.cstart) && up(&c->d_contrib, co.contrib) &&
         up(&c->d_dest, co.dest) && up(&c->d_nd_nodes, co.nd_nodes) &&
         up(&c->d_nd_bnd, co.nd_bnd) && up(&c->d_nd_cmap, co.nd_cmap) && up(&c->d_fw_src, co.fw_src) && up(&c->d_sub_fw_src, co.sub_fw_src) && up(&c->d_fw_items, co.fw_items) &&
         up(&c->d_sub_fw_items, co.sub_fw_items) && up(&c->d_sub_bw_items, co.sub_bw_items) &&
         up(&c->d_sub_fw_off, co.sub_fw_off) && up(&c->d_sub_bw_off, co.sub_bw_off) &&
         up(&c->d_bw_items, co.bw_items) && up(&c->d_lvl_nodes, co.lvl_nodes) &&
         up(&c->d_f_subs, co.f_subs) && up(&c->d_f_nodes, co.f_nodes) && up(&c->d_f_went, co.f_went) &&
         up(&c->d_f_pack, co.f_pack);
}

void build_tables(Ctx* c, std::vector<double>& tab) {
  const int p = c->p, q = c->q, m = c->m;
  Tables& T = c->tab;
  tab.clear();
  auto mark = [&]() { return (int)tab.size(); };
  std::vector<double> gq = gll_points(q);
  // Bernstein gradients at the interpolation points, k3 = a + (q+1) b
  T.off_geo_dN = mark();
  for (int k3 = 0; k3 < c->nL; ++k3) {
    double x1 = gq[k3 % (q + 1)], x2 = gq[k3 / (q + 1)];
    for (int b = 0; b <= m; ++b)
      for (int a = 0; a <= m; ++a) {
        tab.push_back(bernstein_derivative(m, a, x1) * bernstein_value(m, b, x2));
        tab.push_back(bernstein_value(m, a, x1) * bernstein_derivative(m, b, x2));
      }
  }
  // det J check sample: Gauss 2m+2 points plus both ends, tensor product
  std::vector<double> gx, gw;
  gauss_rule(2 * m + 2, gx, gw);
  gx.push_back(0.0);
  gx.push_back(1.0);
  T.off_chk_dN = mark();
  T.nchk = (int)(gx.size() * gx.size());
  for (double x2 : gx)
    for (double x1 : gx)
      for (int b = 0; b <= m; ++b)
        for (int a = 0; a <= m; ++a) {
          tab.push_back(bernstein_derivative(m, a, x1) * bernstein_value(m, b, x2));
          tab.push_back(bernstein_value(m, a, x1) * bernstein_derivative(m, b, x2));
        }
  // edge rule for constraint rows: 2p+2 Gauss points
  std::vector<double> gp = gll_points(p);
  gauss_rule(2 * p + 2, gx, gw);
  T.nq_edge = (int)gx.size();
  T.off_edge_w = mark();
  for (double w : gw) tab.push_back(w);
  T.off_edge_b = mark();
  for (int a = 0; a <= p; ++a)
    for (double x : gx) tab.push_back(lagrange_value(gp, a, x));
  T.off_edge_B = mark();
  for (int a = 0; a <= m; ++a)
    for (double x : gx) tab.push_back(bernstein_value(m, a, x));
  T.off_edge_dB = mark();
  for (int a = 0; a <= m; ++a)
    for (double x : gx) tab.push_back(bernstein_derivative(m, a, x));
  T.off_mid_B = mark();
  for (int a = 0; a <= m; ++a) tab.push_back(bernstein_value(m, a, 0.5));
  T.off_edge_x = mark();
  for (double x : gx) tab.push_back(x);
  T.off_edge_nodes = mark();
  for (double x : gp) tab.push_back(x);
  T.off_edge_bw = mark();
  for (int a = 0; a <= p; ++a) {
    double d = 1.0;
    for (int l = 0; l <= p; ++l)
      if (l != a) d *= gp[a] - gp[l];
    tab.push_back(1.0 / d);
  }
  // load rule: p+2m+2 Gauss points
  gauss_rule(p + 2 * m + 2, gx, gw);
  T.nq_load = (int)gx.size();
  T.off_load_w = mark();
  for (double w : gw) tab.push_back(w);
  T.off_load_b = mark();
  for (int a = 0; a <= p; ++a)
    for (double x : gx) tab.push_back(lagrange_value(gp, a, x));
  T.off_load_dB = mark();
  for (int a = 0; a <= m; ++a)
    for (double x : gx) tab.push_back(bernstein_derivative(m, a, x));
  T.off_load_x = mark();
  for (double x : gx) tab.push_back(x);
  // GLL points of the MDEIM interpolation degree of each family slot
  for (int s = 0; s < 4; ++s) T.off_rnodes[s] = -1;
  for (size_t s = 0; s < c->fam_ids.size() && s < 4; ++s) {
    const RomDev& R = c->roms[c->fam_ids[s]];
    T.off_rnodes[s] = mark();
    for (double v : gll_points(R.r)) tab.push_back(v);
  }
  T.total = (int)tab.size();
}

}  // namespace lbddc
