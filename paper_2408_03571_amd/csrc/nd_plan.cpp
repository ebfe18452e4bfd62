// Host planner for the nested-dissection factorisation of the coarse matrix
// A_0 = R_0 A R_0^T (Sec. 3-4: exact coarse solve).
//
// A_0 is a (2R+1)^2-point operator on the ncx x ncy coarse-unknown grid
// (R = 2 for H = 2h, R = 3 for coarser ratios).  The grid is bisected
// recursively along its longer side by separators R lines wide, which
// decouple the two halves, until boxes are at most `leaf` nodes on a side.
// Every tree node ("front") eliminates its own nodes I (a leaf box or a
// separator) after its two children; its boundary B is the set of
// ancestor-separator nodes within Chebyshev distance R of the node's box,
// which is exactly where the Schur complement of the eliminated box lives.
// Child update matrices (on B_child) are extend-added into the parent front
// F = [I, B] through the index maps built here.
#include <algorithm>
#include <cstdio>
#include <stdexcept>

#include "hs_internal.h"

namespace hs {

namespace {

struct Box {
  int x0, x1, y0, y1;
};

struct Builder {
  int ncx, ncy, R, leaf;
  NDPlan* plan;
  std::vector<Box> seps;        // separator box of each front (or the leaf box)
  std::vector<Box> boxes;       // region box of each front
  std::vector<std::vector<int>> anc;

  int rec(Box b, const std::vector<int>& ancestors, int depth) {
    const int t = (int)plan->fronts.size();
    plan->fronts.push_back(NDFront{});
    boxes.push_back(b);
    seps.push_back(b);
    anc.push_back(ancestors);
    NDFront& f0 = plan->fronts[t];
    f0.depth = depth;
    f0.child[0] = f0.child[1] = -1;
    const int w = b.x1 - b.x0, h = b.y1 - b.y0;
    if (w <= leaf && h <= leaf) return t;
    Box s, c1, c2;
    if (w >= h) {
      const int m = b.x0 + (w - R) / 2;
      s = {m, m + R, b.y0, b.y1};
      c1 = {b.x0, m, b.y0, b.y1};
      c2 = {m + R, b.x1, b.y0, b.y1};
    } else {
      const int m = b.y0 + (h - R) / 2;
      s = {b.x0, b.x1, m, m + R};
      c1 = {b.x0, b.x1, b.y0, m};
      c2 = {b.x0, b.x1, m + R, b.y1};
    }
    seps[t] = s;
    std::vector<int> a2 = ancestors;
    a2.push_back(t);
    const int l = rec(c1, a2, depth + 1);
    const int r = rec(c2, a2, depth + 1);
    plan->fronts[t].child[0] = l;
    plan->fronts[t].child[1] = r;
    return t;
  }
};

}  // namespace

NDPlan build_nd_plan(int ncx, int ncy, int reach, int leaf) {
  if (leaf < reach + 2) leaf = reach + 2;
  NDPlan plan;
  plan.ncx = ncx;
  plan.ncy = ncy;
  plan.reach = reach;
  plan.leaf = leaf;
  Builder b{ncx, ncy, reach, leaf, &plan, {}, {}, {}};
  b.rec(Box{0, ncx, 0, ncy}, {}, 0);
  const int nf = (int)plan.fronts.size();

  // node sets and lookup rectangles
  std::vector<std::vector<int>> Fids(nf);
  for (int t = 0; t < nf; ++t) {
    NDFront& f = plan.fronts[t];
    const Box s = b.seps[t];
    const Box bx = b.boxes[t];
    f.nrect = 0;
    auto add_rect = [&](Box r, int base) {
      if (f.nrect >= kMaxRects) throw std::runtime_error("nested dissection: too many boundary pieces");
      f.rect[f.nrect++] = Rect{r.x0, r.x1, r.y0, r.y1, base};
    };
    // the rectangles first (their bases are running node counts), then the
    // node ids of each in row-major order
    int count = (s.x1 - s.x0) * (s.y1 - s.y0);
    add_rect(s, 0);
    f.nI = count;
    for (int a : b.anc[t]) {
      const Box as = b.seps[a];
      Box r{std::max(as.x0, bx.x0 - reach), std::min(as.x1, bx.x1 + reach),
            std::max(as.y0, bx.y0 - reach), std::min(as.y1, bx.y1 + reach)};
      if (r.x1 <= r.x0 || r.y1 <= r.y0) continue;
      add_rect(r, count);
      count += (r.x1 - r.x0) * (r.y1 - r.y0);
    }
    f.nF = count;
    f.nB = f.nF - f.nI;
    std::vector<int>& ids = Fids[t];
    ids.resize(count);
    for (int q = 0; q < f.nrect; ++q) {
      const Rect& r = f.rect[q];
      int* o = ids.data() + r.base;
      for (int y = r.y0; y < r.y1; ++y)
        for (int x = r.x0; x < r.x1; ++x) *o++ = y * ncx + x;
    }
  }

  // offsets
  {
    size_t nI = 0, nB = 0;
    for (const NDFront& f : plan.fronts) {
      nI += f.nI;
      nB += f.nB;
    }
    plan.Iid.reserve(nI);
    plan.Bid.reserve(nB);
  }
  for (int t = 0; t < nf; ++t) {
    NDFront& f = plan.fronts[t];
    f.Iid = (int64_t)plan.Iid.size();
    plan.Iid.insert(plan.Iid.end(), Fids[t].begin(), Fids[t].begin() + f.nI);
    f.Bid = (int64_t)plan.Bid.size();
    plan.Bid.insert(plan.Bid.end(), Fids[t].begin() + f.nI, Fids[t].end());
    // rows of G and V start on 128-byte boundaries, so a chunk of columns
    // that starts on one reads whole cache lines
    f.ldg = (f.nI + 7) & ~7;
    f.ldv = (f.nB + 7) & ~7;
    f.gofs = plan.g_elems;
    plan.g_elems += (nd_g_entries(f.nI, f.ldg) + 7) & ~(int64_t)7;
    f.vofs = plan.v_elems;
    plan.v_elems += (int64_t)f.nI * f.ldv;
    plan.g_algo += nd_tri(f.nI) ? nd_g_entries(f.nI, f.ldg) : (int64_t)f.nI * f.nI;
    plan.v_algo += (int64_t)f.nI * f.nB;
    f.fofs = plan.f_elems;
    plan.f_elems += (int64_t)f.nF * f.nF;
    f.cofs = plan.c_elems;
    plan.c_elems += f.nI;
    f.uofs = plan.u_elems;
    plan.u_elems += f.nB;
    f.pofs = plan.p_elems;
    plan.p_elems += f.nI;
    plan.max_depth = std::max(plan.max_depth, f.depth);
  }

  // child -> parent positions of every B node (the root has no parent), and
  // the inverse extend-add maps: for parent row r, the child's B index or -1
  // (one map per child of every interior front).  Both are sized once.
  int64_t n_ppos = 0, n_inv = 0;
  for (int t = 0; t < nf; ++t) {
    NDFront& f = plan.fronts[t];
    f.ppofs = n_ppos;
    n_ppos += f.nB;
    f.inv[0] = f.inv[1] = -1;
    if (f.child[0] < 0) continue;
    f.inv[0] = n_inv;
    f.inv[1] = n_inv + f.nF;
    n_inv += 2 * (int64_t)f.nF;
  }
  plan.ppos.assign(n_ppos, -1);
  plan.inv.assign(n_inv, -1);
  // pos[] maps a grid node to its row in the front at hand; it is reset
  // after each front, so the pass costs O(sum of front sizes).
  std::vector<int> pos((size_t)ncx * ncy, -1);
  for (int t = 0; t < nf; ++t) {
    const NDFront& f = plan.fronts[t];
    if (f.child[0] < 0) continue;
    for (int r = 0; r < f.nF; ++r) pos[Fids[t][r]] = r;
    for (int c = 0; c < 2; ++c) {
      const NDFront& fc = plan.fronts[f.child[c]];
      for (int bidx = 0; bidx < fc.nB; ++bidx) {
        const int r = pos[plan.Bid[fc.Bid + bidx]];
        if (r < 0) throw std::runtime_error("nested dissection: child boundary not in parent front");
        plan.inv[f.inv[c] + r] = bidx;
        plan.ppos[fc.ppofs + bidx] = r;
      }
    }
    for (int r = 0; r < f.nF; ++r) pos[Fids[t][r]] = -1;
  }

  plan.levels.assign(plan.max_depth + 1, {});
  for (int t = 0; t < nf; ++t) plan.levels[plan.fronts[t].depth].push_back(t);
  return plan;
}

}  // namespace hs

// ------------------------------------------------------- structural check
extern "C" hs_status hs_nd_plan_check(int ncx, int ncy, int reach, int leaf, int64_t* stats) {
  try {
    if (ncx < 1 || ncy < 1 || reach < 1 || leaf < 1) throw std::runtime_error("bad plan sizes");
    const hs::NDPlan p = hs::build_nd_plan(ncx, ncy, reach, leaf);
    const int nf = (int)p.fronts.size();
    const int64_t N = (int64_t)ncx * ncy;
    // owner front of every node (I sets must partition the grid)
    std::vector<int> owner(N, -1);
    for (int t = 0; t < nf; ++t) {
      const hs::NDFront& f = p.fronts[t];
      for (int r = 0; r < f.nI; ++r) {
        const int g = p.Iid[f.Iid + r];
        if (owner[g] >= 0) throw std::runtime_error("node eliminated twice");
        owner[g] = t;
      }
    }
    for (int64_t g = 0; g < N; ++g)
      if (owner[g] < 0) throw std::runtime_error("node never eliminated");
    // subtree membership via parent links
    std::vector<int> parent(nf, -1);
    for (int t = 0; t < nf; ++t)
      for (int c = 0; c < 2; ++c)
        if (p.fronts[t].child[c] >= 0) parent[p.fronts[t].child[c]] = t;
    auto in_subtree = [&](int t, int node_front) {
      for (int q = node_front; q >= 0; q = parent[q])
        if (q == t) return true;
      return false;
    };
    int64_t st[8] = {nf, p.max_depth + 1, p.g_algo, p.v_algo, p.f_elems, 0, 0, 0};
    for (int t = 0; t < nf; ++t) {
      const hs::NDFront& f = p.fronts[t];
      st[5] = std::max<int64_t>(st[5], f.nI);
      st[6] = std::max<int64_t>(st[6], f.nB);
      st[7] = std::max<int64_t>(st[7], f.nF);
      std::vector<char> expect(N, 0);
      int64_t nexp = 0;
      for (int64_t g = 0; g < N; ++g) {
        if (!in_subtree(t, owner[g])) continue;
        const int gx = (int)(g % ncx), gy = (int)(g / ncx);
        for (int dy = -reach; dy <= reach; ++dy)
          for (int dx = -reach; dx <= reach; ++dx) {
            const int vx = gx + dx, vy = gy + dy;
            if (vx < 0 || vx >= ncx || vy < 0 || vy >= ncy) continue;
            const int64_t v = (int64_t)vy * ncx + vx;
            if (in_subtree(t, owner[v]) || expect[v]) continue;
            expect[v] = 1;
            ++nexp;
          }
      }
      if (nexp != f.nB) throw std::runtime_error("front boundary has the wrong size");
      for (int b = 0; b < f.nB; ++b) {
        const int v = p.Bid[f.Bid + b];
        if (!expect[v]) throw std::runtime_error("front boundary holds a node outside the Schur support");
        // the boundary node must be eliminated later, by an ancestor
        bool anc = false;
        for (int q = parent[t]; q >= 0; q = parent[q]) anc |= (owner[v] == q);
        if (!anc) throw std::runtime_error("front boundary node is not owned by an ancestor");
      }
    }
    // factor layout: each front's G and V blocks start on 128 bytes and lie
    // inside the factor arrays without overlapping another front's; a G kept
    // as one triangle maps (k, c) and (c, k) to one entry and its entries
    // c <= k onto the block one to one
    std::vector<std::pair<int64_t, int64_t>> gb, vb;
    for (const hs::NDFront& f : p.fronts) {
      if ((f.gofs & 7) || (f.vofs & 7)) throw std::runtime_error("factor block not 128-byte aligned");
      if (hs::nd_tri(f.nI)) {
        const int64_t ne = hs::nd_g_entries(f.nI, f.ldg);
        std::vector<char> hit((size_t)ne, 0);
        for (int k = 0; k < f.nI; ++k)
          for (int c = 0; c < f.nI; ++c) {
            const int64_t e = hs::nd_g_index(f.nI, f.ldg, k, c);
            if (e < 0 || e >= ne || e != hs::nd_g_index(f.nI, f.ldg, c, k))
              throw std::runtime_error("triangle of G indexed outside its block or not symmetrically");
            if (c <= k) {
              if (hit[(size_t)e]) throw std::runtime_error("two entries of a triangle of G share a place");
              hit[(size_t)e] = 1;
            }
          }
      }
      gb.push_back({f.gofs, hs::nd_g_entries(f.nI, f.ldg)});
      vb.push_back({f.vofs, (int64_t)f.nI * f.ldv});
    }
    for (auto* blocks : {&gb, &vb}) {
      std::sort(blocks->begin(), blocks->end());
      for (size_t q = 0; q + 1 < blocks->size(); ++q)
        if ((*blocks)[q].first + (*blocks)[q].second > (*blocks)[q + 1].first)
          throw std::runtime_error("factor blocks overlap");
    }
    if (!gb.empty() && (gb.back().first + gb.back().second > p.g_elems || vb.back().first + vb.back().second > p.v_elems))
      throw std::runtime_error("factor block outside the factor array");
    if (stats)
      for (int q = 0; q < 8; ++q) stats[q] = st[q];
    return HS_OK;
  } catch (const std::exception& e) {
    hs::set_error(std::string("nested-dissection plan: ") + e.what());
    return HS_EINVAL;
  }
}
