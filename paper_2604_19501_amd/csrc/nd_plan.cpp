// Symbolic analysis of the exact coarsest-grid solve.
//
// The coarsest operator (eq. 3.6) is a stencil of radius r on a regular node grid:
// 9-point (2D) / 27-point (3D) for the 5/7-point fine operator with full weighting
// (r = 1), 25- or 49-point (2D) and 125-point (3D) for the compact fourth-order stack
// with high-order or level-dependent transfers (r = 2 or 3).  It is solved exactly by
// block Gaussian elimination in a geometric nested-dissection order: a box of nodes is
// cut by a slab of r node planes normal to its longest axis (r planes separate the two
// halves for a stencil of radius r), recursively, until boxes hold at most leaf_max
// nodes.  Every tree node ("front") eliminates its separator S; its boundary B is the
// r-node halo of its box, which lies in ancestor separators.  After its subtree is
// eliminated, a front couples S and B densely.
//
// The separators of the top levels may be merged into one root front (a
// supernode): elimination stays exact, the tree gets shallower, and the solve
// needs fewer dependent steps at the price of a larger dense root block.
//
// This file builds, on the host: the tree, the S/B index lists, the child->parent
// position maps used by the extend-add of Schur complements and their inverses,
// the list of original matrix entries each front assembles, storage offsets, and
// the work schedules of the forward and backward substitutions.
#include <algorithm>
#include <cassert>
#include <cstdio>
#include <functional>
#include <map>
#include <set>
#include <numeric>
#include <stdexcept>

#include "internal.h"

namespace helm {

namespace {

struct Box {
  int lo[3], hi[3];
};

struct Builder {
  Geom g;
  int leaf_max;
  int r = 1;            // stencil radius: separator slab thickness and halo width
  std::vector<Box> box;
  std::vector<std::vector<int>> S, B, kids;
  std::vector<int> parent;

  long long count(const Box& b) const {
    long long c = 1;
    for (int a = 0; a < g.dim; ++a) c *= (b.hi[a] - b.lo[a] + 1);
    return c;
  }
  int flat(int i0, int i1, int i2) const { return i0 + g.N[0] * (i1 + g.N[1] * i2); }

  int build(const Box& b, int par) {
    int id = (int)box.size();
    box.push_back(b);
    S.emplace_back();
    B.emplace_back();
    kids.emplace_back();
    parent.push_back(par);
    int ax = -1, ext = 0;
    for (int a = g.dim - 1; a >= 0; --a) {     // ties: prefer the slowest axis
      int e = b.hi[a] - b.lo[a] + 1;
      if (e > ext) { ext = e; ax = a; }
    }
    bool leaf = count(b) <= leaf_max || ext < r + 2;
    Box sep = b;
    if (!leaf) {
      int mid = (b.lo[ax] + b.hi[ax] - (r - 1)) / 2;     // the slab [mid, mid + r)
      sep.lo[ax] = mid;
      sep.hi[ax] = mid + r - 1;
      Box c0 = b, c1 = b;
      c0.hi[ax] = mid - 1;
      c1.lo[ax] = mid + r;
      int a0 = build(c0, id);
      int a1 = build(c1, id);
      kids[id] = {a0, a1};
    }
    for (int i2 = sep.lo[2]; i2 <= sep.hi[2]; ++i2)
      for (int i1 = sep.lo[1]; i1 <= sep.hi[1]; ++i1)
        for (int i0 = sep.lo[0]; i0 <= sep.hi[0]; ++i0) S[id].push_back(flat(i0, i1, i2));
    // r-node halo of the box inside the domain, increasing flat index
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::max(b.lo[a] - r, 0);
      hi[a] = std::min(b.hi[a] + r, g.N[a] - 1);
    }
    for (int i2 = lo[2]; i2 <= hi[2]; ++i2)
      for (int i1 = lo[1]; i1 <= hi[1]; ++i1)
        for (int i0 = lo[0]; i0 <= hi[0]; ++i0) {
          bool inside = i0 >= b.lo[0] && i0 <= b.hi[0] && i1 >= b.lo[1] && i1 <= b.hi[1] &&
                        i2 >= b.lo[2] && i2 <= b.hi[2];
          if (!inside) B[id].push_back(flat(i0, i1, i2));
        }
    return id;
  }
};

}  // namespace

void nd_plan(const Geom& g3, int leaf_max, int rows_chunk, int root_merge, int elem_bytes, int lds_bytes,
             const std::vector<int>& cuts, long long splitk_bytes, NDPlan& plan, int tree_waves,
             const std::vector<int>& merge_heights, int radius) {
  tree_waves = std::max(1, std::min(16, tree_waves));
  Builder bd;
  bd.g = g3;
  bd.leaf_max = std::max(leaf_max, 1);
  bd.r = std::max(1, radius);
  Box rootbox;
  for (int a = 0; a < 3; ++a) {
    rootbox.lo[a] = 0;
    rootbox.hi[a] = g3.N[a] - 1;
  }
  bd.build(rootbox, -1);
  const int nraw = (int)bd.box.size();
  std::vector<char> alive(nraw, 1);
  // ---- amalgamation: every front whose height in the dissection tree (leaves 0) is listed
  // in merge_heights joins its separator to its parent's, and its children become the
  // parent's.  The parent's box contains the child's, so its boundary is unchanged and the
  // elimination stays exact; the tree loses those levels, at the price of larger fronts.
  if (!merge_heights.empty()) {
    std::vector<int> hraw(nraw, 0), host(nraw);
    for (int t = nraw - 1; t >= 0; --t)        // children have larger ids than their parent
      for (int c : bd.kids[t]) hraw[t] = std::max(hraw[t], hraw[c] + 1);
    std::set<int> mh(merge_heights.begin(), merge_heights.end());
    for (int t = 0; t < nraw; ++t) {
      host[t] = t;
      if (t == 0 || !mh.count(hraw[t])) continue;
      const int q = host[bd.parent[t]];        // resolved first: parents precede children
      bd.S[q].insert(bd.S[q].end(), bd.S[t].begin(), bd.S[t].end());
      alive[t] = 0;
      host[t] = q;
    }
    for (int t = 0; t < nraw; ++t) bd.kids[t].clear();
    for (int t = 1; t < nraw; ++t)
      if (alive[t]) {
        bd.parent[t] = host[bd.parent[t]];
        bd.kids[bd.parent[t]].push_back(t);
      }
    for (int t = 0; t < nraw; ++t)
      if (alive[t]) std::sort(bd.S[t].begin(), bd.S[t].end());
  }
  // ---- merge whole levels of separators into the root while its separator stays <= root_merge
  {
    std::vector<int> frontier = bd.kids[0];
    while (!frontier.empty()) {
      size_t add = 0;
      for (int c : frontier) add += bd.S[c].size();
      if (bd.S[0].size() + add > (size_t)root_merge) break;
      std::vector<int> next;
      for (int c : frontier) {
        bd.S[0].insert(bd.S[0].end(), bd.S[c].begin(), bd.S[c].end());
        alive[c] = 0;
        next.insert(next.end(), bd.kids[c].begin(), bd.kids[c].end());
      }
      frontier = next;
    }
    std::sort(bd.S[0].begin(), bd.S[0].end());
    bd.kids[0] = frontier;
    for (int c : frontier) bd.parent[c] = 0;
  }
  // ---- renumber the surviving fronts (children keep larger ids than their parent)
  std::vector<int> nid(nraw, -1), oid;
  for (int t = 0; t < nraw; ++t)
    if (alive[t]) {
      nid[t] = (int)oid.size();
      oid.push_back(t);
    }
  const int nf = (int)oid.size();
  const long long N3 = g3.tot;
  std::vector<int> owner(N3, -1), pos_in_S(N3, -1);
  for (int t = 0; t < nf; ++t) {
    const std::vector<int>& s = bd.S[oid[t]];
    for (size_t i = 0; i < s.size(); ++i) {
      if (owner[s[i]] != -1) throw std::runtime_error("nd_plan: node in two separators");
      owner[s[i]] = t;
      pos_in_S[s[i]] = (int)i;
    }
  }
  for (long long v = 0; v < N3; ++v)
    if (owner[v] < 0) throw std::runtime_error("nd_plan: node in no separator");
  std::vector<std::vector<int>> kids(nf);
  std::vector<int> par(nf, -1), height(nf, 0);
  for (int t = 0; t < nf; ++t)
    for (int c : bd.kids[oid[t]]) {
      kids[t].push_back(nid[c]);
      par[nid[c]] = t;
    }
  for (int t = nf - 1; t >= 0; --t)
    for (int c : kids[t]) height[t] = std::max(height[t], height[c] + 1);

  plan.g = g3;
  plan.fronts.assign(nf, NDFrontDev());
  plan.idx.clear();
  plan.maps.clear();
  plan.asmv.clear();
  plan.children.clear();
  plan.child_map_off.clear();
  plan.max_height = 0;
  plan.max_children = 0;
  plan.max_nS = plan.max_nB = plan.max_nF = 0;
  long long F = 0, L = 0, W = 0, U = 0, P = 0, La = 0, Wa = 0;
  const long long line = std::max(1, 128 / std::max(1, elem_bytes));   // entries per 128 bytes
  auto pad_ld = [&](long long n) { return (n + line - 1) / line * line; };
  auto Bof = [&](int t) -> const std::vector<int>& { return bd.B[oid[t]]; };
  auto posF = [&](int t, int v) -> int {   // position of node v in front t's (S, B) list, -1 if absent
    if (owner[v] == t) return pos_in_S[v];
    const std::vector<int>& b = Bof(t);
    auto it = std::lower_bound(b.begin(), b.end(), v);
    if (it == b.end() || *it != v) return -1;
    return (int)bd.S[oid[t]].size() + (int)(it - b.begin());
  };
  for (int t = 0; t < nf; ++t) {
    NDFrontDev& f = plan.fronts[t];
    f.nS = (int)bd.S[oid[t]].size();
    f.nB = (int)Bof(t).size();
    f.nF = f.nS + f.nB;
    f.nchild = (int)kids[t].size();
    f.height = height[t];
    plan.max_height = std::max(plan.max_height, f.height);
    plan.max_children = std::max(plan.max_children, f.nchild);
    f.idx_off = (long long)plan.idx.size();
    plan.idx.insert(plan.idx.end(), bd.S[oid[t]].begin(), bd.S[oid[t]].end());
    plan.idx.insert(plan.idx.end(), Bof(t).begin(), Bof(t).end());
    f.F_off = F;  F += (long long)f.nF * f.nF;
    f.ldL = (int)pad_ld(f.nF);
    f.ldW = (int)pad_ld(f.nS);
    f.L_off = La; La += (long long)f.ldL * f.nS;
    f.W_off = Wa; Wa += (long long)f.ldW * f.nB;
    L += (long long)f.nF * f.nS;
    W += (long long)f.nS * f.nB;
    f.upd_off = U; U += f.nB;
    f.perm_off = P; P += f.nS;
    plan.max_nS = std::max(plan.max_nS, f.nS);
    plan.max_nB = std::max(plan.max_nB, f.nB);
    plan.max_nF = std::max(plan.max_nF, f.nF);
  }
  // child -> parent maps (setup extend-add) and, per parent position, the list of
  // child-update entries that add into it (solve gather), as CSR over positions
  plan.cptr.clear();
  plan.cidx.clear();
  for (int t = 0; t < nf; ++t) {
    NDFrontDev& f = plan.fronts[t];
    f.child_off = (int)plan.children.size();
    std::vector<std::vector<int>> contrib(f.nF);
    for (int c = 0; c < f.nchild; ++c) {
      int ch = kids[t][c];
      plan.children.push_back(ch);
      plan.child_map_off.push_back((long long)plan.maps.size());
      std::vector<char> seen(f.nF, 0);
      int k = 0;
      for (int v : Bof(ch)) {
        int p = posF(t, v);
        if (p < 0) throw std::runtime_error("nd_plan: child boundary outside parent front");
        if (seen[p]) throw std::runtime_error("nd_plan: map not injective");
        seen[p] = 1;
        plan.maps.push_back(p);
        long long a = plan.fronts[ch].upd_off + k++;
        if (a > 0x7fffffffLL) throw std::runtime_error("nd_plan: update pool too large");
        contrib[p].push_back((int)a);
      }
    }
    f.inv_off = (long long)plan.cptr.size();
    int acc = (int)plan.cidx.size();
    for (int p = 0; p < f.nF; ++p) {
      plan.cptr.push_back(acc);
      plan.cidx.insert(plan.cidx.end(), contrib[p].begin(), contrib[p].end());
      acc += (int)contrib[p].size();
    }
    plan.cptr.push_back(acc);
  }
  // assembly lists: entry (i, j) of the operator goes to the front where the first
  // eliminated of i, j is a separator node; the other one is then in that front too.
  const int dim = g3.dim;
  const int rr = bd.r, sw = 2 * bd.r + 1;   // stencil radius and width: plane k of offset d
  for (int t = 0; t < nf; ++t) {
    NDFrontDev& f = plan.fronts[t];
    f.asm_off = (long long)plan.asmv.size();
    const Box& bx = bd.box[oid[t]];
    const std::vector<int>& St = bd.S[oid[t]];
    for (int ps = 0; ps < f.nS; ++ps) {
      int s = St[ps];
      int s0 = s % g3.N[0], s1 = (s / g3.N[0]) % g3.N[1], s2 = s / (g3.N[0] * g3.N[1]);
      for (int d2 = (dim == 3 ? -rr : 0); d2 <= (dim == 3 ? rr : 0); ++d2)
        for (int d1 = -rr; d1 <= rr; ++d1)
          for (int d0 = -rr; d0 <= rr; ++d0) {
            int q0 = s0 + d0, q1 = s1 + d1, q2 = s2 + d2;
            if (q0 < 0 || q0 >= g3.N[0] || q1 < 0 || q1 >= g3.N[1] || q2 < 0 || q2 >= g3.N[2]) continue;
            int q = bd.flat(q0, q1, q2);
            int k = (d0 + rr) + sw * (d1 + rr) + (dim == 3 ? sw * sw * (d2 + rr) : 0);
            int kq = (-d0 + rr) + sw * (-d1 + rr) + (dim == 3 ? sw * sw * (-d2 + rr) : 0);
            if (owner[q] == t) {
              plan.asmv.push_back({ps, pos_in_S[q], (long long)k * N3 + s});
            } else {
              bool inbox = q0 >= bx.lo[0] && q0 <= bx.hi[0] && q1 >= bx.lo[1] && q1 <= bx.hi[1] &&
                           q2 >= bx.lo[2] && q2 <= bx.hi[2];
              if (inbox) continue;   // eliminated in a descendant, arrives via extend-add
              int pq = posF(t, q);
              if (pq < 0) throw std::runtime_error("nd_plan: neighbour outside front");
              plan.asmv.push_back({ps, pq, (long long)k * N3 + s});
              plan.asmv.push_back({pq, ps, (long long)kq * N3 + q});
            }
          }
    }
    f.asm_cnt = (int)((long long)plan.asmv.size() - f.asm_off);
  }
  plan.F_total = F;
  plan.L_total = L;
  plan.W_total = W;
  plan.L_alloc = La;
  plan.W_alloc = Wa;
  plan.upd_total = U;
  plan.perm_total = P;
  plan.by_height.assign(plan.max_height + 1, std::vector<int>());
  for (int t = 0; t < nf; ++t) plan.by_height[plan.fronts[t].height].push_back(t);
  // pivot-row buffer of the exchange updates: the rows of one column block (at most
  // ND_KBOUT) of every front of one height
  long long Tmax = 0;
  for (auto& ids : plan.by_height) {
    long long s = 0;
    for (int t : ids) s += (long long)ND_KBOUT * plan.fronts[t].nF;
    Tmax = std::max(Tmax, s);
  }
  plan.T_scratch = Tmax;

  // ---------------- solve schedules ----------------
  // The lower part of the tree runs as tree-block launches: launch (c, b] gives every
  // subtree of fronts with height in (c, b] to one work-group, which walks it level by
  // level (forward ascending, backward descending) with work-group barriers.  Fronts
  // above the last cut run one multi-block launch per height (rows_chunk rows per
  // work-group).  The cuts minimise a cost model of launch and level latencies and of
  // the bandwidth one work-group (tree blocks) or the whole chip (multi-block) can pull.
  const int H = plan.max_height;
  const int KS = 16;                                   // k range of one segment of 64 rows
  auto nparts = [&](int K) { return std::max(1, (K + KS - 1) / KS); };
  auto al16 = [](long long v) { return (v + 15) / 16 * 16; };
  // LDS of one front in a stage: work entries (vector + partials) and schedule bytes
  auto work_entries = [&](const NDFrontDev& f, int dir) -> long long {
    const int R = dir == 0 ? f.nF : f.nS, K = dir == 0 ? f.nS : f.nB;
    if (R == 0 || K == 0) return 0;
    return (long long)(dir == 0 ? f.nF : f.nB) + 64LL * ((R + 63) / 64) * nparts(K);
  };
  auto sched_bytes = [&](const NDFrontDev& f, int dir) -> long long {
    const int R = dir == 0 ? f.nF : f.nS, K = dir == 0 ? f.nS : f.nB;
    if (R == 0 || K == 0) return 0;
    const long long rb = (R + 63) / 64;
    return (long long)sizeof(NDGather) * (dir == 0 ? f.nF : f.nB) + (long long)sizeof(NDSeg) * rb * nparts(K) +
           (long long)sizeof(NDOut) * rb + 4LL * R + (long long)sizeof(NDStage);
  };
  std::vector<double> fbytes(nf);
  for (int t = 0; t < nf; ++t) {
    const NDFrontDev& f = plan.fronts[t];
    fbytes[t] = (double)elem_bytes * ((double)f.nF * f.nS + (double)f.nS * f.nB) + 24.0 * (f.nF + f.nB);
  }
  // launch latency, latency of one level of a tree block (gather, products, outputs and
  // their barriers), bandwidth of one tree-block work-group, of the chip and of one
  // multi-block work-group; per direction
  const double a_launch = 3e-6, a_stage = 5e-6, bw_block = 30e9, bw_chip = 4e12, bw_chunk = 40e9;
  // task root of front t for cut b: its highest ancestor (itself included) of height <= b
  auto task_root = [&](int t, int b) {
    while (par[t] >= 0 && plan.fronts[par[t]].height <= b) t = par[t];
    return t;
  };
  // fronts of heights (c, b] grouped by task; empty if some task does not fit in LDS
  auto group = [&](int c, int b, std::vector<std::vector<int>>& tasks) -> bool {
    tasks.clear();
    std::vector<int> rootid(nf, -1);
    for (int t = 0; t < nf; ++t) {
      int h = plan.fronts[t].height;
      if (h <= c || h > b) continue;
      int r = task_root(t, b);
      if (rootid[r] < 0) {
        rootid[r] = (int)tasks.size();
        tasks.emplace_back();
      }
      tasks[rootid[r]].push_back(t);
    }
    for (auto& tk : tasks)
      for (int dir = 0; dir < 2; ++dir) {
        long long sch = 0, lu = 0;
        std::vector<long long> work(H + 1, 0);
        for (int t : tk) {
          sch += sched_bytes(plan.fronts[t], dir);
          work[plan.fronts[t].height] += work_entries(plan.fronts[t], dir);
          if (dir == 0 && par[t] >= 0 && plan.fronts[par[t]].height <= b) lu += plan.fronts[t].nB;
          if (dir == 0) lu += plan.fronts[t].nF;       // the prefetched right-hand side entries
          // backward: forwarded x_S of in-task ancestors (bound: every front's), prefetched
          // x_B and x_S
          if (dir == 1) lu += 2LL * plan.fronts[t].nS + plan.fronts[t].nB;
        }
        long long wmax = *std::max_element(work.begin(), work.end());
        // (+ the alignment of the LDS areas: up to 15 entries each, and 64 bytes)
        if (al16(sch) + 6 * 16 + 64 + (wmax + lu + 48) * elem_bytes > lds_bytes) return false;
      }
    return !tasks.empty();
  };
  auto cost_tree = [&](int c, int b) -> double {       // +inf if a task does not fit
    std::vector<std::vector<int>> tasks;
    if (!group(c, b, tasks)) return 1e30;
    double tot = 2.0 * a_launch;
    for (int h = c + 1; h <= b; ++h) {
      double mx = 0.0;
      bool any = false;
      for (auto& tk : tasks) {
        double acc = 0.0;
        for (int t : tk)
          if (plan.fronts[t].height == h) {
            acc += fbytes[t];
            any = true;
          }
        mx = std::max(mx, acc);
      }
      if (any) tot += 2.0 * a_stage + mx / bw_block;
    }
    return tot;
  };
  auto cost_chunks = [&](int h) -> double {
    double by = 0.0, blocks = 0.0;
    for (int t : plan.by_height[h]) {
      by += fbytes[t];
      blocks += (plan.fronts[t].nF + rows_chunk - 1) / rows_chunk;
    }
    if (plan.by_height[h].empty()) return 0.0;
    return 2.0 * (a_launch + a_stage) + by / std::min(bw_chip, blocks * bw_chunk);
  };
  std::vector<int> cut;
  if (!cuts.empty()) {
    // requested cuts, ascending, up to the first whose tasks would not fit in LDS
    std::vector<std::vector<int>> tmp;
    for (int c : cuts) {
      if (c < 0 || c > H || (!cut.empty() && c <= cut.back())) continue;
      if (!group(cut.empty() ? -1 : cut.back(), c, tmp)) break;
      cut.push_back(c);
    }
  } else {
    // best[b + 1]: cost of tree-block launches covering heights <= b, from[]: its last cut
    std::vector<double> best(H + 2, 1e30);
    std::vector<int> from(H + 2, -2);
    best[0] = 0.0;
    for (int b = 0; b <= H; ++b)
      for (int c = -1; c < b; ++c) {
        if (best[c + 1] >= 1e29) continue;
        double v = best[c + 1] + cost_tree(c, b);
        if (v < best[b + 1]) {
          best[b + 1] = v;
          from[b + 1] = c;
        }
      }
    std::vector<double> chunks(H + 2, 0.0);        // multi-block launches of heights > e
    for (int h = H; h >= 0; --h) chunks[h] = chunks[h + 1] + cost_chunks(h);
    double bestv = 1e30;
    int beste = -1;
    for (int e = -1; e <= H; ++e) {
      double v = best[e + 1] + chunks[e + 1];
      if (v < bestv) {
        bestv = v;
        beste = e;
      }
    }
    for (int e = beste; e >= 0; e = from[e + 1]) cut.push_back(e);
    std::reverse(cut.begin(), cut.end());
  }
  plan.cuts = cut;

  plan.fwd.clear();
  plan.bwd.clear();
  // front and S position owning each level-3 node (backward tree tasks forward x in LDS)
  std::vector<int> node_front(g3.tot, -1), node_pos(g3.tot, -1);
  for (int t = 0; t < nf; ++t) {
    const NDFrontDev& f = plan.fronts[t];
    for (int i = 0; i < f.nS; ++i) {
      node_front[plan.idx[f.idx_off + i]] = t;
      node_pos[plan.idx[f.idx_off + i]] = i;
    }
  }
  std::vector<NDLaunch> bwd_tree;
  int lo = -1;
  for (int b : cut) {
    std::vector<std::vector<int>> tasks;
    group(lo, b, tasks);
    NDLaunch fl, bl;
    fl.kind = bl.kind = 2;
    fl.threads = bl.threads = 64;
    for (auto& tk : tasks) {
      for (int dir = 0; dir < 2; ++dir) {
        NDLaunch& L = dir == 0 ? fl : bl;
        NDTask T;
        T.st0 = (int)L.stages.size();
        T.g0 = (int)L.gath.size();
        T.s0 = (int)L.segs.size();
        T.o0 = (int)L.outs.size();
        T.d0 = (int)L.dst.size();
        std::vector<std::vector<int>> byh(b + 1);
        for (int u : tk) byh[plan.fronts[u].height].push_back(u);
        long long wmax = 0;
        // forward: the update vectors of fronts whose parent is in the task are also kept in
        // LDS (entries lu_off[u] ..), where the parent's gathers read them
        std::map<int, int> lu_off;
        int nlu = 0;
        // (only fronts that have work in this direction write their outputs; the others'
        // values are read from global memory)
        if (dir == 0) {
          for (int u : tk)
            if (par[u] >= 0 && plan.fronts[par[u]].height <= b && plan.fronts[u].nS > 0 && plan.fronts[u].nB > 0) {
              lu_off[u] = nlu;
              nlu += plan.fronts[u].nB;
            }
        } else {
          // backward: the solution x_S of fronts with a descendant in the task is also kept
          // in LDS (entries lu_off[a] + S position), where the descendants' gathers read it;
          // a front without a boundary has no backward work (its x_S is final already)
          std::set<int> inner;
          for (int u : tk)
            if (par[u] >= 0 && plan.fronts[par[u]].height <= b) inner.insert(par[u]);
          for (int a : inner)
            if (plan.fronts[a].nS > 0 && plan.fronts[a].nB > 0) {
              lu_off[a] = nlu;
              nlu += plan.fronts[a].nS;
            }
        }
        // LDS entry of update index q from a child of f, or -1 when that child is outside
        auto lds_of = [&](const NDFrontDev& f, int q) -> int {
          for (int k = 0; k < f.nchild; ++k) {
            const int c = plan.children[f.child_off + k];
            const NDFrontDev& C = plan.fronts[c];
            if (q >= C.upd_off && q < C.upd_off + C.nB) {
              auto it = lu_off.find(c);
              return it == lu_off.end() ? -1 : it->second + (int)(q - C.upd_off);
            }
          }
          return -1;
        };
        for (int step = 0; step <= b - lo - 1; ++step) {
          const int h = dir == 0 ? lo + 1 + step : b - step;
          NDStage st{(int)L.gath.size() - T.g0, 0, (int)L.segs.size() - T.s0, 0, (int)L.outs.size() - T.o0, 0};
          int vs = 0;
          long long vec_total = 0;
          for (int u : byh[h]) vec_total += work_entries(plan.fronts[u], dir) > 0
                                                ? (dir == 0 ? plan.fronts[u].nF : plan.fronts[u].nB) : 0;
          int ps = (int)vec_total;
          for (int u : byh[h]) {
            const NDFrontDev& f = plan.fronts[u];
            const int R = dir == 0 ? f.nF : f.nS, K = dir == 0 ? f.nS : f.nB;
            if (R == 0 || K == 0) continue;
            const int* ids = plan.idx.data() + f.idx_off;
            if (dir == 0) {
              for (int i = 0; i < f.nF; ++i) {
                int ca = plan.cptr[f.inv_off + i], cb = plan.cptr[f.inv_off + i + 1];
                NDGather g{vs + i, i < f.nS ? ids[i] : -1, -1, -1, 0, 0};
                auto enc = [&](int q) {
                  const int l = lds_of(f, q);
                  return l >= 0 ? -l - 2 : q;
                };
                if (ca < cb) g.u0 = enc(plan.cidx[ca++]);
                if (ca < cb) g.u1 = enc(plan.cidx[ca++]);
                g.ca = ca;
                g.cb = cb;
                L.gath.push_back(g);
              }
            } else {
              for (int j = 0; j < f.nB; ++j) {
                NDGather g{vs + j, ids[f.nS + j], -1, -1, 0, 0};
                const int node = ids[f.nS + j];
                auto it = lu_off.find(node_front[node]);
                if (it != lu_off.end()) g.u0 = -(it->second + node_pos[node]) - 2;
                L.gath.push_back(g);
              }
            }
            for (int r0 = 0; r0 < R; r0 += 64) {
              const int nr = std::min(64, R - r0);
              // a wavefront covers 64 rows x 16 columns, 32 x 32 or 16 x 64
              const int kse = nr <= 16 ? 4 * KS : nr <= 32 ? 2 * KS : KS;
              const int np = std::max(1, (K + kse - 1) / kse);
              for (int p = 0; p < np; ++p) {
                NDSeg sg;
                sg.m_off = dir == 0 ? f.L_off : f.W_off;
                sg.ld = dir == 0 ? f.ldL : f.ldW;
                sg.r0 = r0;
                sg.nr = nr;
                sg.k0 = p * kse;
                sg.k1 = std::min(K, (p + 1) * kse);
                sg.vslot = vs;
                sg.pslot = ps + 64 * p;
                sg.pad = 0;
                L.segs.push_back(sg);
              }
              NDOut ob{r0, nr, vs, ps, np, (int)L.dst.size() - T.d0, 0, 0};
              auto it = lu_off.find(u);
              if (it != lu_off.end()) {
                // forward: row i >= nS -> entry lu_off + i - nS; backward: row i -> lu_off + i
                ob.lu = dir == 0 ? it->second - f.nS + r0 : it->second + r0;
                ob.lu_on = 1;
              }
              L.outs.push_back(ob);
              for (int i = r0; i < r0 + nr; ++i)
                L.dst.push_back(dir == 1 || i < f.nS ? ids[i] : -(int)(f.upd_off + i - f.nS) - 1);
              ps += 64 * np;
            }
            vs += dir == 0 ? f.nF : f.nB;
          }
          st.g1 = (int)L.gath.size() - T.g0;
          st.s1 = (int)L.segs.size() - T.s0;
          st.o1 = (int)L.outs.size() - T.o0;
          wmax = std::max<long long>(wmax, ps);
          if (st.s1 > st.s0) L.stages.push_back(st);
        }
        T.st1 = (int)L.stages.size();
        T.g1 = (int)L.gath.size();
        T.s1 = (int)L.segs.size();
        T.o1 = (int)L.outs.size();
        T.d1 = (int)L.dst.size();
        const long long sch = al16((long long)sizeof(NDStage) * (T.st1 - T.st0)) +
                              al16((long long)sizeof(NDGather) * (T.g1 - T.g0)) +
                              al16((long long)sizeof(NDSeg) * (T.s1 - T.s0)) +
                              al16((long long)sizeof(NDOut) * (T.o1 - T.o0)) + al16(4LL * (T.d1 - T.d0));
        T.nlu = nlu;
        T.pad = 0;
        const long long need = sch +
                               (wmax + nlu + al16(T.g1 - T.g0) + (dir == 1 ? al16(T.d1 - T.d0) : 0)) * elem_bytes +
                               64;
        if (need > lds_bytes) throw std::runtime_error("nd_plan: tree-block task exceeds LDS");
        if (T.st1 > T.st0) {
          L.tasks.push_back(T);
          L.lds_bytes = std::max<int>(L.lds_bytes, (int)need);
          // wavefronts: one per segment of the widest stage, at most 16
          const int per = 1;
          for (int st = T.st0; st < T.st1; ++st) {
            const int ns = L.stages[st].s1 - L.stages[st].s0;
            L.threads = std::max(L.threads, 64 * std::min(tree_waves, (ns + per - 1) / per));
          }
        }
      }
    }
    fl.task_off.assign(1, 0);
    bl.task_off.assign(1, 0);
    plan.fwd.push_back(fl);
    bwd_tree.push_back(bl);
    lo = b;
  }
  std::vector<NDLaunch> bwd_high;
  const int KT = 128;                                  // columns of a split-K tile
  auto build_splitk = [&](NDLaunch& L, int h, int dir) {
    L.kind = 3;
    for (int t : plan.by_height[h]) {
      const NDFrontDev& f = plan.fronts[t];
      const int R = dir == 0 ? f.nF : f.nS, K = dir == 0 ? f.nS : f.nB;
      if (R == 0 || K == 0) continue;
      const int* ids = plan.idx.data() + f.idx_off;
      const int voff = (int)L.gath.size();
      if (dir == 0) {
        for (int i = 0; i < f.nF; ++i) {
          int ca = plan.cptr[f.inv_off + i], cb = plan.cptr[f.inv_off + i + 1];
          NDGather g{voff + i, i < f.nS ? ids[i] : -1, -1, -1, 0, 0};
          if (ca < cb) g.u0 = plan.cidx[ca++];
          if (ca < cb) g.u1 = plan.cidx[ca++];
          g.ca = ca;
          g.cb = cb;
          L.gath.push_back(g);
        }
      } else {
        for (int j = 0; j < f.nB; ++j) L.gath.push_back({voff + j, ids[f.nS + j], -1, -1, 0, 0});
      }
      const int nkt = (K + KT - 1) / KT;
      for (int r0 = 0; r0 < R; r0 += 256) {
        const int ps0 = (int)L.p_elems;
        for (int kt = 0; kt < nkt; ++kt) {
          L.tiles.push_back({t, r0, kt * KT, std::min(K, (kt + 1) * KT), (int)L.p_elems, voff});
          L.p_elems += 256;
        }
        L.rtiles.push_back({t, r0, nkt, ps0, voff, 0});
      }
    }
  };
  for (int h = lo + 1; h <= plan.max_height; ++h) {
    NDLaunch fl, bl;
    fl.kind = bl.kind = 1;
    fl.task_off.push_back(0);
    bl.task_off.push_back(0);
    long long bf = 0, bb = 0;
    for (int t : plan.by_height[h]) {
      bf += (long long)plan.fronts[t].nF * plan.fronts[t].nS * elem_bytes;
      bb += (long long)plan.fronts[t].nS * plan.fronts[t].nB * elem_bytes;
    }
    if (bf >= splitk_bytes) {
      build_splitk(fl, h, 0);
    } else {
      for (int t : plan.by_height[h]) {
        const NDFrontDev& f = plan.fronts[t];
        // the front's gather list: row i reads r at its node (i < nS) and the children's
        // updates, the first two inline
        const int g0 = (int)fl.gath.size();
        const int* ids = plan.idx.data() + f.idx_off;
        for (int i = 0; i < f.nF; ++i) {
          int ca = plan.cptr[f.inv_off + i];
          const int cb = plan.cptr[f.inv_off + i + 1];
          NDGather g{i, i < f.nS ? ids[i] : -1, -1, -1, 0, 0};
          if (ca < cb) g.u0 = plan.cidx[ca++];
          if (ca < cb) g.u1 = plan.cidx[ca++];
          g.ca = ca;
          g.cb = cb;
          fl.gath.push_back(g);
        }
        for (int r = 0; r < f.nF; r += rows_chunk) {
          fl.items.push_back({t, r, std::min(f.nF, r + rows_chunk), h, f.nS, f.nF, f.nB, g0, f.ldL, 0, f.L_off, f.idx_off,
                              f.inv_off, f.upd_off});
          fl.task_off.push_back((int)fl.items.size());
        }
        fl.max_rows_vec = std::max(fl.max_rows_vec, f.nF);
      }
    }
    if (bb >= splitk_bytes && bb > 0) {
      build_splitk(bl, h, 1);
    } else {
      for (int t : plan.by_height[h]) {
        const NDFrontDev& f = plan.fronts[t];
        if (f.nB > 0)          // a front without boundary has nothing to back-substitute
          for (int r = 0; r < f.nS; r += rows_chunk) {
            bl.items.push_back({t, r, std::min(f.nS, r + rows_chunk), h, f.nS, f.nF, f.nB, 0, f.ldW, 0, f.W_off, f.idx_off,
                                f.inv_off, f.upd_off});
            bl.task_off.push_back((int)bl.items.size());
          }
        bl.max_rows_vec = std::max(bl.max_rows_vec, f.nB);
      }
    }
    plan.fwd.push_back(fl);
    if (!bl.items.empty() || !bl.tiles.empty()) bwd_high.push_back(bl);
  }
  std::vector<NDLaunch> bwd_all(bwd_high.rbegin(), bwd_high.rend());
  for (auto it = bwd_tree.rbegin(); it != bwd_tree.rend(); ++it)
    if (!it->tasks.empty()) bwd_all.push_back(*it);
  plan.bwd = bwd_all;
}


}  // namespace helm
