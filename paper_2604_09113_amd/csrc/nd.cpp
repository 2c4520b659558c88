// Nested-dissection symbolic analysis of the coarse problem S_C (host side,
// integer topology only).
//
// Coarse dofs sit on grid vertices (2 values) and cell edges (averages and
// moment).  Placing them at doubled coordinates (vertex (2vx, 2vy), horizontal
// edge (2ex+1, 2vy), vertical edge (2vx, 2ey+1)), the cell grid is bisected
// recursively across its longer side; the dofs on each cutting grid line
// (inside the box, not taken by an ancestor) form that node's separator, and
// boxes of at most 2 x 2 cells are leaves that own their remaining dofs.
// Two coarse dofs couple only through a shared cell, so every node couples only
// to dofs of its own box, and its front is [own dofs | box dofs owned by
// ancestors].  Each entry of S_C is summed into the front of the deeper of the
// two owning nodes (the one that eliminates first).
#include <algorithm>
#include <map>

#include "internal.h"

namespace lbddc {

namespace {

struct Obj {
  int X, Y, first, size, owner;
};

struct Builder {
  int nx, ny;
  std::vector<Obj> objs;
  std::vector<int> at;  // (2ny+1) x (2nx+1) -> object index or -1
  std::vector<NDNodeH> nodes;
  std::vector<std::vector<int>> own_objs;
  std::vector<std::array<int, 4>> box;

  int lookup(int X, int Y) const { return at[(size_t)Y * (2 * nx + 1) + X]; }

  int build(int x0, int x1, int y0, int y1, int parent, int depth) {
    const int id = (int)nodes.size();
    nodes.push_back(NDNodeH());
    own_objs.push_back({});
    box.push_back({x0, x1, y0, y1});
    nodes[id].parent = parent;
    nodes[id].level = depth;
    const int w = x1 - x0, h = y1 - y0;
    const bool leaf = std::max(w, h) <= 2;
    int cut = -1;
    bool vertical = w >= h;
    if (!leaf) cut = vertical ? (x0 + x1) / 2 : (y0 + y1) / 2;
    std::vector<int> mine;
    for (int Y = 2 * y0; Y <= 2 * y1; ++Y)
      for (int X = 2 * x0; X <= 2 * x1; ++X) {
        int o = lookup(X, Y);
        if (o < 0 || objs[o].owner >= 0) continue;
        if (leaf || (vertical ? X == 2 * cut : Y == 2 * cut)) mine.push_back(o);
      }
    for (int o : mine) objs[o].owner = id;
    own_objs[id] = mine;
    if (!leaf) {
      int c0, c1;
      if (vertical) {
        c0 = build(x0, cut, y0, y1, id, depth + 1);
        c1 = build(cut, x1, y0, y1, id, depth + 1);
      } else {
        c0 = build(x0, x1, y0, cut, id, depth + 1);
        c1 = build(x0, x1, cut, y1, id, depth + 1);
      }
      nodes[id].child[0] = c0;
      nodes[id].child[1] = c1;
    }
    return id;
  }
};

}  // namespace

bool build_nested_dissection(Ctx* c, const std::vector<int>& ent_g1, const std::vector<int>& ent_g2) {
  const int nx = c->nx, ny = c->ny, nce = c->nce;
  CoarseLayout& co = c->co;
  Builder B;
  B.nx = nx;
  B.ny = ny;
  B.at.assign((size_t)(2 * nx + 1) * (2 * ny + 1), -1);
  auto add = [&](int X, int Y, int first, int size) {
    B.at[(size_t)Y * (2 * nx + 1) + X] = (int)B.objs.size();
    B.objs.push_back({X, Y, first, size, -1});
  };
  // vertices and edges on clamped sides carry no coarse dof and are no objects
  for (int vy = 0; vy <= ny; ++vy)
    for (int vx = 0; vx <= nx; ++vx) {
      const int f = co.vert_first[(size_t)vy * (nx + 1) + vx];
      if (f >= 0) add(2 * vx, 2 * vy, f, 2);
    }
  for (int vy = 0; vy <= ny; ++vy)
    for (int ex = 0; ex < nx; ++ex) {
      const int f = co.hedge_first[(size_t)vy * nx + ex];
      if (f >= 0) add(2 * ex + 1, 2 * vy, f, nce);
    }
  for (int ey = 0; ey < ny; ++ey)
    for (int vx = 0; vx <= nx; ++vx) {
      const int f = co.vedge_first[(size_t)ey * (nx + 1) + vx];
      if (f >= 0) add(2 * vx, 2 * ey + 1, f, nce);
    }
  B.build(0, nx, 0, ny, -1, 0);
  const int nn = (int)B.nodes.size();
  // own and boundary dof lists, front positions
  std::vector<int> owner_of_dof(c->NC, -1);
  for (auto& o : B.objs)
    for (int k = 0; k < o.size; ++k) owner_of_dof[o.first + k] = o.owner;
  for (int o = 0; o < (int)B.objs.size(); ++o)
    if (B.objs[o].owner < 0) {
      c->err = "internal: a coarse dof without a nested-dissection owner";
      return false;
    }
  auto is_ancestor = [&](int a, int n) {  // a is a strict ancestor of n
    for (int p = B.nodes[n].parent; p >= 0; p = B.nodes[p].parent)
      if (p == a) return true;
    return false;
  };
  co.nd_own.clear();
  co.nd_bnd.clear();
  co.nd_cmap.clear();
  std::vector<std::vector<int>> own(nn), bnd(nn);
  for (int n = 0; n < nn; ++n) {
    std::vector<int> oo = B.own_objs[n];
    std::sort(oo.begin(), oo.end(), [&](int a, int b) { return B.objs[a].first < B.objs[b].first; });
    for (int o : oo)
      for (int k = 0; k < B.objs[o].size; ++k) own[n].push_back(B.objs[o].first + k);
    const auto& bx = B.box[n];
    std::vector<int> bo;
    for (int Y = 2 * bx[2]; Y <= 2 * bx[3]; ++Y)
      for (int X = 2 * bx[0]; X <= 2 * bx[1]; ++X) {
        int o = B.lookup(X, Y);
        if (o >= 0 && is_ancestor(B.objs[o].owner, n)) bo.push_back(o);
      }
    std::sort(bo.begin(), bo.end(), [&](int a, int b) { return B.objs[a].first < B.objs[b].first; });
    for (int o : bo)
      for (int k = 0; k < B.objs[o].size; ++k) bnd[n].push_back(B.objs[o].first + k);
  }
  // node table, levels, storage offsets
  co.nd_nodes.assign(nn, NDNodeH());
  co.nd_levels.clear();
  long long foff = 0;
  int ooff = 0, boff = 0, uoff = 0, eoff = 0;
  co.nd_nfmax = 0;
  co.nd_nsmax = 0;
  for (int n = 0; n < nn; ++n) {
    NDNodeH& d = co.nd_nodes[n];
    d = B.nodes[n];
    d.ns = (int)own[n].size();
    d.nb = (int)bnd[n].size();
    d.foff = foff;
    foff += (long long)(d.ns + d.nb) * (d.ns + d.nb);
    d.own_off = ooff;
    ooff += d.ns;
    d.bnd_off = boff;
    boff += d.nb;
    d.up_off = uoff;
    uoff += d.nb;
    d.beff_off = eoff;
    eoff += d.ns;
    co.nd_nfmax = std::max(co.nd_nfmax, d.ns + d.nb);
    co.nd_nsmax = std::max(co.nd_nsmax, d.ns);
    co.nd_own.insert(co.nd_own.end(), own[n].begin(), own[n].end());
    co.nd_bnd.insert(co.nd_bnd.end(), bnd[n].begin(), bnd[n].end());
    if ((int)co.nd_levels.size() <= d.level) co.nd_levels.resize(d.level + 1);
    co.nd_levels[d.level].push_back(n);
  }
  co.nd_front_total = foff;
  // pivot-column panels of the levels swept in blocks (fronts above ND_LDS_NF)
  co.nd_cp_total = 0;
  for (const auto& lv : co.nd_levels) {
    int nfmax = 0;
    for (int n : lv) nfmax = std::max(nfmax, co.nd_nodes[n].ns + co.nd_nodes[n].nb);
    if (nfmax <= ND_LDS_NF) continue;
    long long off = 0;
    for (int n : lv) {
      co.nd_nodes[n].cp_off = off;
      off += 64LL * (co.nd_nodes[n].ns + co.nd_nodes[n].nb);
    }
    co.nd_cp_total = std::max(co.nd_cp_total, off);
  }
  co.nd_up_total = uoff;
  co.nd_beff_total = eoff;
  // child maps: child bnd position -> parent front position
  for (int n = 0; n < nn; ++n) {
    NDNodeH& d = co.nd_nodes[n];
    for (int s = 0; s < 2; ++s) {
      int ch = d.child[s];
      d.cmap_off[s] = -1;
      if (ch < 0) continue;
      d.cmap_off[s] = (int)co.nd_cmap.size();
      for (int g : bnd[ch]) {
        int pos = -1;
        auto it = std::find(own[n].begin(), own[n].end(), g);
        if (it != own[n].end()) pos = (int)(it - own[n].begin());
        else {
          auto jt = std::find(bnd[n].begin(), bnd[n].end(), g);
          if (jt != bnd[n].end()) pos = d.ns + (int)(jt - bnd[n].begin());
        }
        if (pos < 0) {
          c->err = "internal: a child boundary dof missing from its parent front";
          return false;
        }
        co.nd_cmap.push_back(pos);
      }
    }
  }
  // destinations of the S_C entries: front of the deeper owner
  co.dest.assign(ent_g1.size(), 0);
  std::vector<int> posn(c->NC, -1);  // scratch: position in the front currently indexed
  // group entries by the node whose front receives them
  std::vector<int> tgt(ent_g1.size());
  for (size_t e = 0; e < ent_g1.size(); ++e) {
    int a = owner_of_dof[ent_g1[e]], b = owner_of_dof[ent_g2[e]];
    tgt[e] = (a == b || is_ancestor(b, a)) ? a : b;
  }
  std::vector<std::vector<int>> by_node(nn);
  for (size_t e = 0; e < ent_g1.size(); ++e) by_node[tgt[e]].push_back((int)e);
  for (int n = 0; n < nn; ++n) {
    const NDNodeH& d = co.nd_nodes[n];
    const int nf = d.ns + d.nb;
    for (int i = 0; i < d.ns; ++i) posn[own[n][i]] = i;
    for (int i = 0; i < d.nb; ++i) posn[bnd[n][i]] = d.ns + i;
    for (int e : by_node[n]) {
      int p1 = posn[ent_g1[e]], p2 = posn[ent_g2[e]];
      if (p1 < 0 || p2 < 0) {
        c->err = "internal: a coarse matrix entry outside its front";
        return false;
      }
      co.dest[e] = d.foff + (long long)p1 * nf + p2;
    }
    for (int g : own[n]) posn[g] = -1;
    for (int g : bnd[n]) posn[g] = -1;
  }
  return true;
}

}  // namespace lbddc

namespace lbddc {

// Program of the fused bottom-level forward sweep (FusedSub): every subtree
// rooted at level L - ND_FUSED_LEVELS gets its packed M^T rows, the vector
// entries of each node (where every front position of w comes from) and the
// offsets of its nodes in LDS.  Sets co.fused only when every subtree fits
// (single row part per node, LDS, entry and pair budgets); otherwise the
// per-level kernels and the three-level subtree kernel are used.
void build_fused_sweeps(Ctx* c) {
  CoarseLayout& co = c->co;
  co.fused = false;
  co.f_subs.clear(); co.f_nodes.clear(); co.f_went.clear(); co.f_pack.clear();
  co.f_blk_total = 0;
  const int L = (int)co.nd_levels.size();
  const int ls = L - ND_FUSED_LEVELS;
  if (ls < 0 || (int)co.nd_levels[ls].size() < ND_FUSED_MIN_ROOTS) return;
  for (int l = ls; l < L; ++l)
    for (int n : co.nd_levels[l])
      if (co.nd_nodes[n].ns > ND_KPART) return;
  long long total = 0;
  std::vector<FusedSub> subs;
  std::vector<FusedNode> fnodes;
  std::vector<short4> went;
  std::vector<FusedPack> pack;
  for (int root : co.nd_levels[ls]) {
    // the subtree's nodes by depth below the root
    std::vector<std::vector<int>> by(ND_FUSED_LEVELS);
    std::vector<int> stack{root};
    while (!stack.empty()) {
      const int n = stack.back();
      stack.pop_back();
      const int d = co.nd_nodes[n].level - ls;
      if (d < 0 || d >= ND_FUSED_LEVELS) return;
      by[d].push_back(n);
      for (int s = 1; s >= 0; --s)
        if (co.nd_nodes[n].child[s] >= 0) stack.push_back(co.nd_nodes[n].child[s]);
    }
    for (auto& v : by) std::sort(v.begin(), v.end());
    FusedSub S{};
    // own dofs: one contiguous range (tree order)
    int lo = 1 << 30, tot = 0;
    for (auto& v : by)
      for (int n : v) { lo = std::min(lo, co.nd_nodes[n].own_off); tot += co.nd_nodes[n].ns; }
    for (auto& v : by)
      for (int n : v)
        if (co.nd_nodes[n].own_off + co.nd_nodes[n].ns > lo + tot) return;
    S.own_off = lo;
    S.own_n = tot;
    S.node0 = (int)fnodes.size();
    std::map<int, int> slot;  // node id -> index in fnodes
    int mt = 0, vec = 0;
    for (int d = 0; d < ND_FUSED_LEVELS; ++d) {
      S.stage_node[d] = (int)fnodes.size() - S.node0;
      if ((int)by[d].size() > ND_FUSED_STAGE_NODES) return;
      S.stage_pairs[d] = 0;
      for (int n : by[d]) {
        const NDNodeH& D = co.nd_nodes[n];
        FusedNode f{};
        f.pair0 = S.stage_pairs[d];
        S.stage_pairs[d] += D.nb;
        f.ns = D.ns; f.nb = D.nb; f.nf = D.ns + D.nb;
        f.mt = mt; mt += D.ns * D.nb;
        f.w = vec; vec += f.nf;
        f.up = vec; vec += D.nb;
        f.own = D.own_off - lo;
        f.gup = d == 0 ? D.up_off : -1;
        slot[n] = (int)fnodes.size();
        fnodes.push_back(f);
        pack.push_back(FusedPack{D.foff, 0, D.ns, D.nb});
      }
      if (S.stage_pairs[d] > ND_FUSED_THREADS) return;
    }
    S.stage_node[ND_FUSED_LEVELS] = (int)fnodes.size() - S.node0;
    if ((int)fnodes.size() - S.node0 > 16) return;
    S.fwd_n = (mt + 1) & ~1;
    S.vec_n = (vec + 1) & ~1;
    S.fwd_off = total;
    total += S.fwd_n;
    // budgets: LDS, 16-byte loads per thread, one own value per thread
    if ((long long)S.fwd_n + S.vec_n + S.own_n > ND_FUSED_LDS_DOUBLES) return;
    if (S.fwd_n / 2 > ND_FUSED_LOADS * ND_FUSED_THREADS) return;
    if (S.own_n > ND_FUSED_THREADS || S.vec_n >= 32767) return;
    // vector entries by depth: own right-hand side and the children's up
    // vectors (the child map gives the front position of each child boundary
    // entry)
    for (int d = 0; d < ND_FUSED_LEVELS; ++d) {
      S.went[d] = (int)went.size();
      for (int n : by[d]) {
        const NDNodeH& D = co.nd_nodes[n];
        const FusedNode& f = fnodes[slot[n]];
        const size_t first = went.size();
        for (int j = 0; j < D.ns + D.nb; ++j) {
          short4 e;
          e.x = (short)(f.w + j);
          e.y = e.z = -1;
          e.w = (short)(j < D.ns ? f.own + j : -1);
          went.push_back(e);
        }
        for (int s = 0; s < 2; ++s) {
          const int ch = D.child[s];
          if (ch < 0) continue;
          const NDNodeH& C = co.nd_nodes[ch];
          const FusedNode& fc = fnodes[slot.at(ch)];
          for (int i = 0; i < C.nb; ++i) {
            const int pos = co.nd_cmap[D.cmap_off[s] + i];
            short4& e = went[first + pos];
            (s == 0 ? e.y : e.z) = (short)(fc.up + i);
          }
        }
      }
    }
    S.went[ND_FUSED_LEVELS] = (int)went.size();
    if (S.went[ND_FUSED_LEVELS] - S.went[0] > ND_FUSED_ENT * ND_FUSED_THREADS) return;
    subs.push_back(S);
  }
  {
    size_t k = 0;
    for (const FusedSub& S : subs)
      for (int i = 0; i < S.stage_node[ND_FUSED_LEVELS]; ++i, ++k) pack[k].fdst = S.fwd_off + fnodes[S.node0 + i].mt;
  }
  co.f_subs = std::move(subs);
  co.f_nodes = std::move(fnodes);
  co.f_went = std::move(went);
  co.f_pack = std::move(pack);
  co.f_blk_total = total;
  co.fused_level = ls;
  co.fused = true;
}

}  // namespace lbddc
