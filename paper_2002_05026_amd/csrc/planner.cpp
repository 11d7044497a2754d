// Host planner for the dual block LDL^T of D3M (Sec. II of the paper).
//
// The paper builds its task graph by symbolically simulating the sequential
// algorithm and then maps the weighted graph onto processors with a list
// scheduling heuristic (Sec. II).  Here the same simulation produces the
// DAG of tile tasks for one GPU, and a list scheduler over the persistent
// workgroups turns bottom-level priorities into the ticket order in which
// workgroups take tasks.  The schedule only orders tickets: correctness
// comes from the device-side dependency counters.
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
#include <map>
#include <set>
#include <unordered_map>

namespace d3m {

// ----------------------------------------------------------------- geometry
// Interfaces of an a x b x c domain grid (axis 0 first, then 1, then 2; the
// lower domain's coordinates x slowest, z fastest); interface (ax, d)
// separates domains d and d + e_ax.
std::vector<std::array<int32_t, 4>> grid_interfaces(const int32_t* g) {
  std::vector<std::array<int32_t, 4>> out;
  for (int ax = 0; ax < 3; ++ax)
    for (int x = 0; x < g[0]; ++x)
      for (int y = 0; y < g[1]; ++y)
        for (int z = 0; z < g[2]; ++z) {
          int up[3] = {x, y, z};
          up[ax]++;
          if (up[0] < g[0] && up[1] < g[1] && up[2] < g[2]) out.push_back({ax, x, y, z});
        }
  return out;
}

namespace {
void nd_rec(const std::vector<std::array<int32_t, 4>>& f, std::array<int, 3> lo,
            std::array<int, 3> hi, std::vector<int32_t>& out) {
  int e[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
  if (e[0] * e[1] * e[2] <= 1) return;
  int ax = (e[1] > e[0]) ? 1 : 0;
  if (e[2] > e[ax]) ax = 2;
  int cut = lo[ax] + e[ax] / 2;
  auto mid_hi = hi, mid_lo = lo;
  mid_hi[ax] = cut;
  mid_lo[ax] = cut;
  nd_rec(f, lo, mid_hi, out);
  nd_rec(f, mid_lo, hi, out);
  for (size_t i = 0; i < f.size(); ++i) {
    if (f[i][0] != ax || f[i][1 + ax] != cut - 1) continue;
    bool inside = true;
    for (int t = 0; t < 3; ++t) {
      int c0 = f[i][1 + t], c1 = c0 + (t == ax ? 1 : 0);
      if (c0 < lo[t] || c1 >= hi[t]) inside = false;
    }
    if (inside) out.push_back((int32_t)i);
  }
}
}  // namespace

// Nested dissection over the domain grid: cut the longest box axis (ties to
// the lowest axis) in the middle; order = low half, high half, separator.
std::vector<int32_t> nd_order(const int32_t* grid) {
  auto f = grid_interfaces(grid);
  std::vector<int32_t> out;
  nd_rec(f, {0, 0, 0}, {grid[0], grid[1], grid[2]}, out);
  return out;
}

// Greedy minimum degree on the block graph (with fill), ties by id.
std::vector<int32_t> min_degree_order(int nb, const std::vector<std::array<int32_t, 2>>& pairs) {
  std::vector<std::set<int>> adj(nb);
  for (auto& pr : pairs) {
    adj[pr[0]].insert(pr[1]);
    adj[pr[1]].insert(pr[0]);
  }
  std::vector<char> done(nb, 0);
  std::vector<int32_t> out;
  for (int step = 0; step < nb; ++step) {
    int best = -1;
    size_t bd = SIZE_MAX;
    for (int i = 0; i < nb; ++i)
      if (!done[i] && adj[i].size() < bd) { bd = adj[i].size(); best = i; }
    done[best] = 1;
    out.push_back(best);
    std::vector<int> nb_(adj[best].begin(), adj[best].end());
    for (int a : nb_) adj[a].erase(best);
    for (size_t u = 0; u < nb_.size(); ++u)
      for (size_t v = u + 1; v < nb_.size(); ++v) {
        adj[nb_[u]].insert(nb_[v]);
        adj[nb_[v]].insert(nb_[u]);
      }
    adj[best].clear();
  }
  return out;
}

// ----------------------------------------------------------------- schedule
namespace {

struct GenDag {
  std::vector<Task> t;
  std::vector<std::vector<int32_t>> preds;
  std::vector<double> w;  // estimated microseconds
  int add(const Task& task, std::vector<int32_t> pr, double weight) {
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    pr.erase(std::remove(pr.begin(), pr.end(), -1), pr.end());
    t.push_back(task);
    preds.push_back(std::move(pr));
    w.push_back(std::max(weight, 0.5));
    return (int)t.size() - 1;
  }
};

// List scheduling of a weighted DAG on P identical workers with bottom-level
// priority; the ticket order is the simulated start order.
void finalize(GenDag& g, int P, int sched, TaskDag& out) {
  const int n = (int)g.t.size();
  std::vector<std::vector<int32_t>> succ(n);
  for (int i = 0; i < n; ++i)
    for (int p : g.preds[i]) succ[p].push_back(i);
  std::vector<double> bl(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double m = 0;
    for (int s : succ[i]) m = std::max(m, bl[s]);
    bl[i] = g.w[i] + m;
  }
  std::vector<double> start(n, 0.0);
  double makespan = 0;
  if (sched == 1) {
    for (int i = 0; i < n; ++i) start[i] = i;
  } else {
    std::vector<int> indeg(n);
    auto cmp = [&](int a, int b) { return bl[a] < bl[b] || (bl[a] == bl[b] && a > b); };
    std::priority_queue<int, std::vector<int>, decltype(cmp)> ready(cmp);
    for (int i = 0; i < n; ++i) {
      indeg[i] = (int)g.preds[i].size();
      if (indeg[i] == 0) ready.push(i);
    }
    typedef std::pair<double, int> Ev;
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> ev;
    int free_w = std::max(P, 1);
    double now = 0;
    int done = 0;
    while (done < n) {
      while (free_w > 0 && !ready.empty()) {
        int t = ready.top();
        ready.pop();
        start[t] = now;
        ev.push({now + g.w[t], t});
        --free_w;
      }
      if (ev.empty()) break;  // cycle (cannot happen for a generated DAG)
      Ev e = ev.top();
      ev.pop();
      now = e.first;
      ++free_w;
      ++done;
      for (int s : succ[e.second])
        if (--indeg[s] == 0) ready.push(s);
    }
    makespan = now;
  }
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (start[a] != start[b]) return start[a] < start[b];
    if (bl[a] != bl[b]) return bl[a] > bl[b];
    return a < b;
  });
  std::vector<int> ticket(n);
  for (int i = 0; i < n; ++i) ticket[ord[i]] = i;
  out.tasks.resize(n);
  out.npred.resize(n);
  out.gen_of.resize(n);
  out.succ.clear();
  for (int k = 0; k < n; ++k) {
    int i = ord[k];
    Task t = g.t[i];
    t.succ_begin = (int32_t)out.succ.size();
    std::vector<int32_t> s;
    for (int q : succ[i]) s.push_back(ticket[q]);
    std::sort(s.begin(), s.end());
    for (int q : s) out.succ.push_back(q);
    t.nsucc = (int32_t)s.size();
    out.tasks[k] = t;
    out.npred[k] = (int32_t)g.preds[i].size();
    out.gen_of[k] = i;
  }
  out.gpreds = std::move(g.preds);
  out.weight_us = g.w;
  out.makespan_us = makespan;
}

// Task durations (microseconds) used only to weight the list schedule,
// fitted to traces of the complex64 tasks on MI355X.  A tile product costs a
// fixed part (task start, first slab, store) plus its executed MFMA work:
// rows count as 64 up to 64 rows and as 128 above (waves per SIMD), columns
// as 16, 64 or 128 (the accumulator widths).
double tile_work(double m, double n, double k) {
  const double me = m > 64 ? 128 : 64, ne = n > 64 ? 128 : (n > 16 ? 64 : 16);
  return 8.0 * me * ne * k;
}
double w_gemm(double m, double n, double k) { return 22.0 + tile_work(m, n, k) / 5.5e5; }
double w_trsm(double m, double n, double k) { return 23.0 + tile_work(m, n, k) / 4.2e5; }
double w_fact(double n) {
  const double r = n / 128.0;
  return 23.0 + 28.5 * r * r * r + 97.0 * r;
}
// solve tasks: weighted for 64 right-hand sides
double w_solve(double m, double k) { return 22.0 + tile_work(m, 64, k) / 5.5e5; }

int64_t key3(int64_t panel, int64_t g, int64_t c) { return (panel << 40) | (g << 12) | c; }

}  // namespace

// ----------------------------------------------------------------- the plan
std::string build_plan(PlanImpl& p, int nb, const int32_t* sizes, int64_t npair, const int32_t* pairs,
                       const int32_t* order, const int32_t* grid, int tile, int nworkers, int sched, int nelim,
                       int solve_tile, int merge, int rhs_groups, int* err) {
  *err = -1;  // D3M_ERR_ARG
  if (nb <= 0 || !sizes || npair < 0 || (npair > 0 && !pairs)) return "bad sizes or pairs";
  if (tile == 0) tile = 128;
  if (tile < 16 || tile > kTileMax || tile % 16) return "tile must be a multiple of 16 in [16,128]";
  p.tile = tile;
  if (solve_tile == 0) solve_tile = 64;
  if (solve_tile < 16 || solve_tile > kTileMax || solve_tile % 16) return "solve_tile must be a multiple of 16 in [16,128]";
  p.solve_tile = solve_tile;
  if (merge == 0) merge = 8;
  if (merge < 1 || merge > kMergeSrc) return "merge must be in [1, 16]";
  p.merge = merge;
  if (rhs_groups == 0) rhs_groups = 1;
  if (rhs_groups < 1 || rhs_groups > 8) return "rhs_groups must be in [1, 8]";
  p.rhs_groups = rhs_groups;
  p.nworkers = nworkers > 0 ? nworkers : 256;
  p.sched = sched;
  p.nb = nb;
  p.n.assign(sizes, sizes + nb);
  for (int i = 0; i < nb; ++i)
    if (sizes[i] < 1) return "interface size must be >= 1";
  *err = -2;  // D3M_ERR_PATTERN
  std::set<std::pair<int, int>> seen;
  for (int64_t k = 0; k < npair; ++k) {
    int a = pairs[2 * k], b = pairs[2 * k + 1];
    if (a < 0 || b < 0 || a >= nb || b >= nb) return "pair id out of range";
    if (a == b) return "self pair";
    auto key = std::make_pair(std::min(a, b), std::max(a, b));
    if (!seen.insert(key).second) return "duplicate pair";
    p.pairs.push_back({std::max(a, b), std::min(a, b)});
  }
  // K offsets: diagonal blocks, then pairs in the given order
  p.koff.assign(nb + npair + 1, 0);
  for (int i = 0; i < nb; ++i) p.koff[i + 1] = p.koff[i] + (int64_t)p.n[i] * p.n[i];
  for (int64_t k = 0; k < npair; ++k)
    p.koff[nb + k + 1] = p.koff[nb + k] + (int64_t)p.n[p.pairs[k][0]] * p.n[p.pairs[k][1]];
  // elimination order
  std::vector<int32_t> ord;
  if (order) {
    ord.assign(order, order + nb);
  } else if (grid) {
    if (grid[0] < 1 || grid[1] < 1 || grid[2] < 1) return "bad grid";
    if ((int)grid_interfaces(grid).size() != nb) return "grid interface count differs from nblk";
    ord = nd_order(grid);
  } else {
    ord = min_degree_order(nb, p.pairs);
  }
  std::vector<int32_t> chk(ord);
  std::sort(chk.begin(), chk.end());
  for (int i = 0; i < nb; ++i)
    if ((int)chk.size() != nb || chk[i] != i) return "order is not a permutation";
  p.order = ord;
  p.pos.assign(nb, 0);
  for (int k = 0; k < nb; ++k) p.pos[ord[k]] = k;
  // partial elimination: the first nelim blocks of the order are eliminated,
  // the others must be the user ids 0..nred-1, and the pairs between them
  // must come first in the pair list
  if (nelim < 0 || nelim >= nb) {
    if (nelim != 0) return "nelim must be in [0, nblk)";
  }
  p.nelim = nelim;
  p.nred = nelim > 0 ? nb - nelim : 0;
  if (nelim > 0) {
    for (int k = nelim; k < nb; ++k)
      if (ord[k] >= p.nred) return "the blocks left after a partial elimination must be the user ids 0..nred-1";
    int64_t npr = 0;
    while (npr < npair && p.pairs[npr][0] < p.nred && p.pairs[npr][1] < p.nred) ++npr;
    for (int64_t k = npr; k < npair; ++k)
      if (p.pairs[k][0] < p.nred && p.pairs[k][1] < p.nred)
        return "the pairs between the blocks left must come first";
    p.npair_red = (int)npr;
  }
  // block fill by elimination in position space
  std::vector<std::set<int>> adj(nb);
  for (auto& pr : p.pairs) {
    int a = p.pos[pr[0]], b = p.pos[pr[1]];
    adj[a].insert(b);
    adj[b].insert(a);
  }
  p.S.assign(nb, {});
  for (int I = 0; I < nb; ++I) {
    std::vector<int32_t> later;
    for (int J : adj[I])
      if (J > I) later.push_back(J);
    for (size_t u = 0; u < later.size(); ++u)
      for (size_t v = u + 1; v < later.size(); ++v) {
        adj[later[u]].insert(later[v]);
        adj[later[v]].insert(later[u]);
      }
    p.S[I] = later;  // std::set iteration is sorted
  }
  if (nelim > 0) {
    // eliminating the leading blocks must create no block between the others
    // that is not in the pair list (the reduced matrix keeps K's layout)
    std::set<std::pair<int, int>> red;
    for (int k = 0; k < p.npair_red; ++k) red.insert({p.pairs[k][0], p.pairs[k][1]});
    for (int I = 0; I < nelim; ++I)
      for (size_t u = 0; u < p.S[I].size(); ++u)
        for (size_t v = 0; v < u; ++v) {
          const int a = p.order[p.S[I][u]], b = p.order[p.S[I][v]];
          if (a >= p.nred || b >= p.nred) continue;
          if (!red.count({std::max(a, b), std::min(a, b)}))
            return "a partial elimination fills a block between the blocks left that is not a pair";
        }
  }
  // counts and flops (8 real flops per complex multiply-add)
  p.L_blocks = 0;
  p.nnz_L = 0;
  p.nnz_K = 0;
  std::vector<int> height(nb, 1);
  p.etree_height = 0;
  p.max_S = 0;
  auto nn = [&](int position) { return (double)p.n[p.order[position]]; };
  const int nfac = nelim > 0 ? nelim : nb;  // panels eliminated
  for (int I = 0; I < nb; ++I) {
    double nI = nn(I);
    p.nnz_L += (int64_t)nI * ((int64_t)nI + 1) / 2;
    if (I >= nfac) continue;
    p.flops_diag += 4.0 / 3.0 * nI * nI * nI;
    p.L_blocks += p.S[I].size();
    p.max_S = std::max(p.max_S, (int)p.S[I].size());
    for (size_t u = 0; u < p.S[I].size(); ++u) {
      double nJ = nn(p.S[I][u]);
      p.nnz_L += (int64_t)nJ * (int64_t)nI;
      p.flops_trsm += 4.0 * nJ * nI * nI;
      p.flops_update += 4.0 * nJ * nJ * nI;
      for (size_t v = 0; v < u; ++v) p.flops_update += 8.0 * nJ * nn(p.S[I][v]) * nI;
    }
    p.etree_height = std::max(p.etree_height, height[I]);
    if (!p.S[I].empty()) height[p.S[I][0]] = std::max(height[p.S[I][0]], height[I] + 1);
  }
  if (nelim > 0) {
    int64_t orig_in = 0;  // pairs stored in an eliminated panel
    for (auto& pr : p.pairs)
      if (std::min(p.pos[pr[0]], p.pos[pr[1]]) < nelim) ++orig_in;
    p.fill_blocks = p.L_blocks - orig_in;
  } else {
    p.fill_blocks = p.L_blocks - npair;
  }
  for (int i = 0; i < nb; ++i) p.nnz_K += (int64_t)p.n[i] * (p.n[i] + 1) / 2;
  for (auto& pr : p.pairs) p.nnz_K += (int64_t)p.n[pr[0]] * p.n[pr[1]];

  // ---- panels, row blocks, tiles
  p.panels.assign(nb, Panel());
  p.pblocks.clear();
  p.tiles.clear();
  int64_t prow0 = 0, loff = 0, linv = 0;
  std::vector<std::unordered_map<int, int>> prow_in(nb);  // panel -> (J -> prow)
  for (int I = 0; I < nb; ++I) {
    Panel& P = p.panels[I];
    int nI = p.n[p.order[I]];
    P.n = nI;
    P.user = p.order[I];
    P.prow0 = (int32_t)prow0;
    P.pb0 = (int32_t)p.pblocks.size();
    int h = 0;
    std::vector<int> rowlist{I};
    for (int J : p.S[I]) rowlist.push_back(J);
    for (int J : rowlist) {
      PBlock b;
      b.J = J;
      b.prow = h;
      b.n = p.n[p.order[J]];
      b.prow0 = 0;  // filled below once all prow0 are known
      prow_in[I][J] = h;
      p.pblocks.push_back(b);
      // blocks start at even rows and the panel height is even, so every
      // tile column of L and LD starts 16-byte aligned in complex64 (the
      // engine's direct LDS loads need it); an odd block leaves one unused row
      h += b.n + (b.n & 1);
    }
    P.npb = (int32_t)rowlist.size();
    P.H = h;
    P.off = loff;
    loff += (int64_t)h * nI;
    P.ioff = linv;
    linv += (int64_t)nI * nI;
    // tiles: nt = ceil(n/T), all of size T but the last.  A tile product
    // costs the same MFMA time for any row count in (64, 128] (8 waves of 16
    // rows, two per SIMD) and any column count in (64, 128], so full tiles
    // and one short remainder (which costs half when it is 64 or less) take
    // less MFMA time than near-equal sizes: n = 300 as 128+128+44 costs
    // 128+128+64 rows against 3*128 for 112+112+76.
    int nt = (nI + tile - 1) / tile;
    int base = tile;
    P.tile0 = (int32_t)p.tiles.size();
    P.nt = nt;
    for (int c = 0; c < nt; ++c) {
      Tile t;
      t.panel = I;
      t.r0 = c * base;
      t.sz = (c == nt - 1) ? nI - c * base : base;
      t.pad = 0;
      t.linv_off = P.ioff + t.r0 + (int64_t)t.r0 * nI;
      p.tiles.push_back(t);
    }
    prow0 += nI;
  }
  p.N = prow0;
  p.L_elems = loff;
  p.Linv_elems = linv;
  for (auto& b : p.pblocks) b.prow0 = p.panels[b.J].prow0;
  for (auto& t : p.tiles)
    if (t.sz <= 0) { *err = -1; return "internal tiling error"; }

  // ---- K placement (scatter) and fill blocks
  p.kplace.clear();
  p.fills.clear();
  for (int i = 0; i < nb; ++i) {
    int I = p.pos[i];
    const Panel& P = p.panels[I];
    p.kplace.push_back({p.koff[i], P.off, P.n, P.n, P.H, 0, i, i});
  }
  std::set<std::pair<int, int>> orig;  // (row panel J, col panel I), J > I
  for (size_t k = 0; k < p.pairs.size(); ++k) {
    int a = p.pairs[k][0], b = p.pairs[k][1];  // K_ab stored, n_a x n_b
    int pa = p.pos[a], pb = p.pos[b];
    if (pa > pb) {  // block (a, b) lives in panel b at rows of a: copy as is
      const Panel& P = p.panels[pb];
      p.kplace.push_back({p.koff[nb + k], P.off + prow_in[pb][pa], p.n[a], p.n[b], P.H, 0, a, b});
      orig.insert({pa, pb});
    } else {        // block (b, a) = K_ab^T lives in panel a at rows of b
      const Panel& P = p.panels[pa];
      p.kplace.push_back({p.koff[nb + k], P.off + prow_in[pa][pb], p.n[b], p.n[a], P.H, 1, b, a});
      orig.insert({pb, pa});
    }
  }
  std::vector<std::pair<int, int>> fill_of;  // (row panel J, col panel I) of each fill block
  for (int I = 0; I < nb; ++I)
    for (int J : p.S[I])
      if (!orig.count({J, I})) {
        const Panel& P = p.panels[I];
        p.fills.push_back({P.off + prow_in[I][J], p.n[p.order[J]], P.n, P.H});
        fill_of.push_back({J, I});
      }

  // ---- residual block rows (user numbering)
  p.rrow.assign(nb, {});
  for (int i = 0; i < nb; ++i) p.rrow[i].push_back({p.koff[i], i, 0});
  for (size_t k = 0; k < p.pairs.size(); ++k) {
    int a = p.pairs[k][0], b = p.pairs[k][1];
    p.rrow[a].push_back({p.koff[nb + k], b, 1});  // K_ab x_b
    p.rrow[b].push_back({p.koff[nb + k], a, 2});  // K_ab^T x_a
  }

  // ---- factor DAG (symbolic simulation of the sequential elimination)
  // Per panel I, a tiled right-looking LDL^T: FACT of each diagonal tile,
  // TRSM of every row tile below it inside the panel, IUPD of the panel's
  // remaining columns; then XUPD of every tile of the blocks (J, K), J, K in
  // S_I, with the whole panel width as inner dimension.
  GenDag g;
  std::vector<std::vector<Access>> facc;
  std::unordered_map<int64_t, int> lastw;  // storage tile -> last writer
  // tiles of each fill block whose first writer stores its product (no K
  // entries there to add it to), keyed by (row panel, col panel)
  std::map<std::pair<int, int>, int> fill_first;
  auto lw = [&](int64_t k) { auto it = lastw.find(k); return it == lastw.end() ? -1 : it->second; };
  const int64_t kDKey = 1LL << 61;
  auto inv_key = [](int64_t a, int64_t b) { return (1LL << 59) | (a << 20) | b; };
  const bool want_acc = true;
  // Updates of one target tile from consecutive source panels are merged
  // into one XUPD task (up to kMergeSrc sources, run one after the other
  // into one accumulator), so the target is read and written once per group
  // and the fixed cost of a task is paid once.  A group waits in pend until
  // it is full or its target panel comes up for elimination.
  struct PendUpd {
    Task t;
    std::vector<int32_t> pr;
    std::vector<Access> ac;
    std::vector<XSrc> src;
    double w;
  };
  std::unordered_map<int64_t, PendUpd> pend;
  std::vector<std::vector<int64_t>> pend_of(nb);  // target panel -> keys possibly pending
  auto emit_upd = [&](int64_t tk, PendUpd& pu) {
    Task t = pu.t;
    if (pu.src.size() > 1) {
      t.pad0 = (int32_t)pu.src.size();
      t.pad1 = (int32_t)p.xsrc.size();
      t.k = 0;
      for (auto& x : pu.src) {
        p.xsrc.push_back(x);
        t.k += x.k;
      }
    }
    int id = g.add(t, pu.pr, pu.w);
    lastw[tk] = id;
    if (want_acc) facc.push_back(pu.ac);
  };
  for (int I = 0; I < nb; ++I) {
    const Panel& P = p.panels[I];
    const int nI = P.n;
    // updates still waiting for more sources whose target is this panel
    for (int64_t tk : pend_of[I]) {
      auto it = pend.find(tk);
      if (it == pend.end()) continue;
      emit_upd(tk, it->second);
      pend.erase(it);
    }
    pend_of[I].clear();
    if (I >= nfac) continue;  // left with its Schur complement (partial elimination)
    // row tiles of the panel: (global tile index, row offset in panel)
    std::vector<std::pair<int, int>> rows;
    for (int b = 0; b < P.npb; ++b) {
      const PBlock& B = p.pblocks[P.pb0 + b];
      const Panel& PJ = p.panels[B.J];
      for (int r = 0; r < PJ.nt; ++r) rows.push_back({PJ.tile0 + r, B.prow + p.tiles[PJ.tile0 + r].r0});
    }
    std::vector<int> trsm_last(rows.size(), -1);  // last TRSM of each row tile
    for (int c = 0; c < P.nt; ++c) {
      const Tile& TC = p.tiles[P.tile0 + c];
      // FACT(I, c)
      Task f{};
      f.kind = TK_FACT;
      f.panel = I;
      f.m = f.n = f.k = TC.sz;
      f.lda = P.H;
      f.aux = P.tile0 + c;
      f.dofs = P.prow0 + TC.r0;
      f.a_off = P.off + TC.r0 + (int64_t)TC.r0 * P.H;
      const int64_t kcc = key3(I, P.tile0 + c, c);
      int fid = g.add(f, {lw(kcc)}, w_fact(TC.sz));
      lastw[kcc] = fid;
      if (want_acc) facc.push_back({{kcc, true}, {inv_key(P.tile0 + c, P.tile0 + c), true}, {kDKey | (P.tile0 + c), true}});
      // TRSM(I, r, c) for every row tile after c
      std::vector<int> trsm(rows.size(), -1);
      for (size_t r = c + 1; r < rows.size(); ++r) {
        const Tile& TR = p.tiles[rows[r].first];
        Task t{};
        t.kind = TK_TRSM;
        t.panel = I;
        t.m = TR.sz;
        t.n = t.k = TC.sz;
        t.lda = P.H;
        t.aux = P.tile0 + c;
        t.dofs = P.prow0 + TC.r0;
        t.a_off = P.off + rows[r].second + (int64_t)TC.r0 * P.H;
        t.b_off = TC.linv_off;
        t.ldc = nI;  // leading dimension of the inverse block
        const int64_t krc = key3(I, rows[r].first, c);
        int tid = g.add(t, {fid, lw(krc)}, w_trsm(TR.sz, TC.sz, TC.sz));
        lastw[krc] = tid;
        trsm[r] = tid;
        trsm_last[r] = tid;
        if (want_acc)
          facc.push_back({{krc, true}, {inv_key(P.tile0 + c, P.tile0 + c), false}, {kDKey | (P.tile0 + c), false}});
      }
      // IUPD(I, r, s, c): A_rs -= L_rc D_c L_sc^T, s a later tile of I, r >= s
      for (int s2 = c + 1; s2 < P.nt; ++s2) {
        const Tile& TS = p.tiles[P.tile0 + s2];
        for (size_t r = s2; r < rows.size(); ++r) {
          const Tile& TR = p.tiles[rows[r].first];
          Task u{};
          u.kind = TK_XUPD;
          u.panel = I;
          u.m = TR.sz;
          u.n = TS.sz;
          u.k = TC.sz;
          u.lda = P.H;
          u.ldc = P.H;
          u.dofs = P.prow0 + TC.r0;
          u.aux = ((int)r == s2) ? 1 : 0;
          u.a_off = P.off + rows[r].second + (int64_t)TC.r0 * P.H;
          u.b_off = P.off + rows[s2].second + (int64_t)TC.r0 * P.H;
          u.c_off = P.off + rows[r].second + (int64_t)TS.r0 * P.H;
          const int64_t krs = key3(I, rows[r].first, s2);
          int uid = g.add(u, {trsm[r], trsm[s2], lw(krs)}, w_gemm(TR.sz, TS.sz, TC.sz));
          lastw[krs] = uid;
          if (want_acc)
            facc.push_back({{krs, true}, {key3(I, rows[r].first, c), false}, {key3(I, rows[s2].first, c), false},
                            {kDKey | (P.tile0 + c), false}});
        }
      }
    }
    // INV(I, r, c): tile (r, c) of the inverse of the unit lower diagonal
    // block, Linv_rc = -Linv_rr sum_{c <= q < r} L_rq Linv_qc; only the
    // solve needs it, so nothing in the factor waits for it
    {
      std::vector<int> fact_of(P.nt);
      for (int c = 0; c < P.nt; ++c) fact_of[c] = lw(key3(I, P.tile0 + c, c));
      for (int c = 0; c < P.nt; ++c) {
        const Tile& TC = p.tiles[P.tile0 + c];
        int prev = -1;
        for (int r = c + 1; r < P.nt; ++r) {
          const Tile& TR = p.tiles[P.tile0 + r];
          Task v{};
          v.kind = TK_INV;
          v.panel = I;
          v.m = TR.sz;
          v.n = TC.sz;
          v.k = TR.r0 - TC.r0;
          v.aux = P.tile0 + r;
          v.dofs = P.tile0 + c;
          std::vector<int32_t> pr{fact_of[r], fact_of[c], prev};
          int vid = g.add(v, pr, w_gemm(TC.sz, TR.sz, TR.r0 - TC.r0) + w_gemm(TR.sz, TC.sz, TR.sz));
          prev = vid;
          if (want_acc) {
            std::vector<Access> ac{{inv_key(P.tile0 + r, P.tile0 + c), true},
                                   {inv_key(P.tile0 + c, P.tile0 + r), true},
                                   {inv_key(P.tile0 + r, P.tile0 + r), false}};
            for (int q = c; q < r; ++q) {
              ac.push_back({key3(I, P.tile0 + r, q), false});
              ac.push_back({inv_key(P.tile0 + q, P.tile0 + c), false});
            }
            facc.push_back(ac);
          }
        }
      }
    }
    // XUPD: A_JK -= L_JI D_I L_KI^T, tile by tile, J >= K in S_I
    const int own = P.nt;
    for (int u = 1; u < P.npb; ++u) {
      const PBlock& BJ = p.pblocks[P.pb0 + u];
      const Panel& PJ = p.panels[BJ.J];
      for (int v = 1; v <= u; ++v) {
        const PBlock& BK = p.pblocks[P.pb0 + v];
        const Panel& PK = p.panels[BK.J];
        const int rowJinK = prow_in[BK.J][BJ.J];
        for (int r = 0; r < PJ.nt; ++r)
          for (int s2 = 0; s2 < PK.nt; ++s2) {
            if (u == v && r < s2) continue;
            const Tile& TR = p.tiles[PJ.tile0 + r];
            const Tile& TS = p.tiles[PK.tile0 + s2];
            // index of the row tiles in this panel's row list
            int ri = -1, si = -1;
            for (size_t q = own; q < rows.size(); ++q) {
              if (rows[q].first == PJ.tile0 + r) ri = (int)q;
              if (rows[q].first == PK.tile0 + s2) si = (int)q;
            }
            Task t{};
            t.kind = TK_XUPD;
            t.panel = I;
            t.m = TR.sz;
            t.n = TS.sz;
            t.k = nI;
            t.lda = P.H;
            t.ldc = PK.H;
            t.dofs = P.prow0;
            t.aux = (u == v && r == s2) ? 1 : 0;
            t.a_off = P.off + BJ.prow + TR.r0;
            t.b_off = P.off + BK.prow + TS.r0;
            t.c_off = PK.off + rowJinK + TR.r0 + (int64_t)TS.r0 * PK.H;
            int64_t tk = key3(BK.J, PJ.tile0 + r, s2);
            auto it = pend.find(tk);
            // in the last sixteenth of the order (the dense top of the tree,
            // whose panels form a chain) a source is not merged behind
            // earlier ones: their product runs while this panel is still
            // being factored, and the target waits for this panel's only
            // (measured: the last eighth, quarter or half do less well, the
            // last 24th or 32nd about as well).  Plans of fewer than
            // kChainMin interfaces keep merging: their chains are short, and
            // in a batch other instances fill the time
            if (it != pend.end() && nb >= kChainMin && 16 * I >= 15 * nb) {
              emit_upd(tk, it->second);
              pend.erase(it);
              it = pend.end();
            }
            if (it == pend.end()) {
              PendUpd pu;
              pu.t = t;
              pu.pr = {lw(tk)};
              if (pu.pr[0] < 0 && u != v && !orig.count({BJ.J, BK.J})) {
                pu.t.aux |= 2;  // the tile's first update, in a fill block: store, not add
                ++fill_first[{BJ.J, BK.J}];
              }
              pu.ac = {{tk, true}};
              pu.w = 22.0;
              it = pend.emplace(tk, std::move(pu)).first;
              pend_of[BK.J].push_back(tk);
            }
            PendUpd& pu = it->second;
            pu.pr.push_back(trsm_last[ri]);
            pu.pr.push_back(trsm_last[si]);
            pu.src.push_back({t.a_off, t.b_off, nI, P.H});
            pu.w += tile_work(TR.sz, TS.sz, nI) / 5.5e5 + (pu.src.size() > 1 ? 3.0 : 0.0);
            if (want_acc)
              for (int c = 0; c < P.nt; ++c) {
                pu.ac.push_back({key3(I, PJ.tile0 + r, c), false});
                pu.ac.push_back({key3(I, PK.tile0 + s2, c), false});
                pu.ac.push_back({kDKey | (P.tile0 + c), false});
              }
            if ((int)pu.src.size() >= p.merge) {
              emit_upd(tk, pu);
              pend.erase(it);
            }
          }
      }
    }
  }
  finalize(g, p.nworkers, sched, p.fdag);
  if (g.t.size() <= 40000) p.facc = std::move(facc);
  // a fill block every tile of which is first written by an update that
  // stores its product needs no zeroing; only its padding row (after an odd
  // last row, read with it as a row pair) does, zeroed with the row before
  // it as one aligned pair (that row's value is stored by its update later)
  {
    std::vector<PlanImpl::FillPlace> keep;
    for (size_t f = 0; f < p.fills.size(); ++f) {
      const auto& F = p.fills[f];
      const auto it = fill_first.find(fill_of[f]);
      const int ntile = p.panels[fill_of[f].first].nt * p.panels[fill_of[f].second].nt;
      if (it == fill_first.end() || it->second < ntile) keep.push_back(F);
      else if (F.rows & 1) keep.push_back({F.dst + F.rows - 1, 2, F.cols, F.ld_dst});
    }
    p.fills = std::move(keep);
  }

  // ---- solve DAG: forward (elimination order), then backward (reverse).
  // W holds b (then x), Z holds z = D^-1 L^-1 b (then t); the diagonal
  // blocks are applied through their precomputed inverses.  The solve cuts
  // each factor tile into row tiles of at most solve_tile rows: a solve task
  // has only nrhs columns, and a 64-row task keeps one wave per SIMD busy in
  // about half the time of a 128-row one, which shortens the chains of
  // updates into one tile that bound the solve.  Solve tiles never cross a
  // factor tile: the tile rows of Linv_II are only valid left of the end of
  // their factor tile (the upper tiles serve the INV tasks as staging).
  const int kSolveTile = p.solve_tile;
  std::vector<int> st0(nb + 1, 0);  // solve tiles of panel I: st0[I] .. st0[I+1]-1
  std::vector<std::pair<int, int>> stl;  // (r0, sz)
  std::vector<std::pair<int, int>> stf;  // (first row, end) of the factor tile holding each solve tile
  for (int I = 0; I < nb; ++I) {
    const Panel& P = p.panels[I];
    for (int c = 0; c < P.nt; ++c) {
      const Tile& T = p.tiles[P.tile0 + c];
      const int nt = (T.sz + kSolveTile - 1) / kSolveTile;
      for (int q = 0; q < nt; ++q) {
        // even starts (16-byte aligned operand columns, as for the factor tiles)
        const int r0 = (T.sz * q / nt) & ~1, r1 = q + 1 == nt ? T.sz : (T.sz * (q + 1) / nt) & ~1;
        stl.push_back({T.r0 + r0, r1 - r0});
        stf.push_back({T.r0, T.r0 + T.sz});
      }
    }
    st0[I + 1] = (int)stl.size();
  }
  std::vector<std::vector<std::pair<int, int>>> holders(nb);  // J -> (panel I, row offset of J in I)
  for (int I = 0; I < nb; ++I)
    for (int b = 1; b < p.panels[I].npb; ++b) {
      const PBlock& B = p.pblocks[p.panels[I].pb0 + b];
      holders[B.J].push_back({I, B.prow});
    }
  const int64_t kWKey = 1LL << 60, kZKey = 1LL << 58;
  // The right-hand sides may be split into G groups of columns: the solve
  // DAG is then G independent copies, copy g working on columns
  // [g ceil(nrhs/G), (g+1) ceil(nrhs/G)) (its group is kept in bits 8.. of
  // the task kind).  Twice the tasks of half the length: twice the
  // parallelism and half as long dependency chains.
  struct GState {
    std::vector<int> lastb, lastz, nupd;
    std::vector<std::vector<int>> ftile, btile;
    std::vector<std::array<int, kSolveSlots + 1>> lastx;
    struct PendF {
      Task t;
      std::vector<int32_t> pr;
      std::vector<Access> ac;
      std::vector<XSrc> src;
      double w = 22.0;
    };
    std::vector<PendF> pendf;
  };
  auto gen_solve = [&](int G, TaskDag& fwd_out, std::vector<std::vector<Access>>& fwd_acc, TaskDag* bwd_out,
                       std::vector<std::vector<Access>>* bwd_acc) {
    GenDag sg, sgb;
    std::vector<std::vector<Access>> sacc, saccb;
    const bool split = bwd_out != nullptr;  // backward part as a launch of its own
    GenDag& bg = split ? sgb : sg;
    std::vector<std::vector<Access>>& bacc = split ? saccb : sacc;
    const double wn = std::max(16, 64 / G);  // columns per task, for the weights
    auto wsolve = [&](double m, double k) { return 22.0 + tile_work(m, wn, k) / 5.5e5; };
    std::vector<GState> gs(G);
    for (auto& q : gs) {
      q.lastb.assign(stl.size(), -1);
      q.lastz.assign(stl.size(), -1);
      q.nupd.assign(stl.size(), 0);
      q.ftile.assign(nb, {});
      q.btile.assign(nb, {});
      q.lastx.resize(stl.size());
      for (auto& a : q.lastx) a.fill(-1);
      q.pendf.assign(stl.size(), GState::PendF());
    }
    auto forward = [&](int g) {
      GState& S = gs[g];
      const int64_t gk = (int64_t)g << 50;
      auto wkey = [&](int slot, int r) { return kWKey | gk | ((int64_t)slot << 40) | r; };
      // forward updates into tile r go round-robin to b and its extra
      // accumulators (count of updates so far, last task per extra slot)
      auto emit_fupd = [&](int r) {
        GState::PendF& pf = S.pendf[r];
        if (pf.src.empty()) return;
        const int slot = S.nupd[r]++ % (kSolveSlots + 1);
        Task u = pf.t;
        u.c_off += (int64_t)slot * p.N;                    // rows of b_r (or a copy) in W
        u.n = (slot > 0 && S.lastx[r][slot] < 0) ? 1 : 0;  // first into a copy: overwrite
        if (pf.src.size() > 1) {
          u.pad0 = (int32_t)pf.src.size();
          u.pad1 = (int32_t)p.xsrc.size();
          u.k = 0;
          for (auto& x : pf.src) {
            p.xsrc.push_back(x);
            u.k += x.k;
          }
        }
        std::vector<int32_t> pr = pf.pr;
        pr.push_back(slot == 0 ? S.lastb[r] : S.lastx[r][slot]);
        std::vector<Access> ac = pf.ac;
        ac[0] = {wkey(slot, r), true};
        int uid = sg.add(u, pr, pf.w);
        if (slot == 0) S.lastb[r] = uid;
        else S.lastx[r][slot] = uid;
        sacc.push_back(ac);
        pf = GState::PendF();
      };
      for (int I = 0; I < nb; ++I) {
        const Panel& P = p.panels[I];
        for (int c = st0[I]; c < st0[I + 1]; ++c) emit_fupd(c);
        // sum the extra accumulators of I's tiles into b_I
        for (int c = st0[I]; c < st0[I + 1]; ++c) {
          const int used = std::min(S.nupd[c], kSolveSlots + 1) - 1;
          if (used <= 0) continue;
          Task t{};
          t.kind = TK_RED | (g << 8);
          t.panel = I;
          t.m = stl[c].second;
          t.k = used;
          t.aux = c;
          t.c_off = P.prow0 + stl[c].first;
          std::vector<int32_t> pr{S.lastb[c]};
          std::vector<Access> ac{{wkey(0, c), true}};
          for (int q = 1; q <= used; ++q) {
            pr.push_back(S.lastx[c][q]);
            ac.push_back({wkey(q, c), false});
          }
          S.lastb[c] = sg.add(t, pr, 10.0);
          sacc.push_back(ac);
        }
        if (I >= nfac) continue;  // not eliminated: its rows now hold the reduced right-hand side
        std::vector<int32_t> inpr;
        for (int c = st0[I]; c < st0[I + 1]; ++c) inpr.push_back(S.lastb[c]);
        for (int c = st0[I]; c < st0[I + 1]; ++c) {
          const int r0 = stl[c].first, sz = stl[c].second;
          Task t{};
          t.kind = TK_FTILE | (g << 8);
          t.panel = I;
          t.m = sz;
          t.k = r0 + sz;
          t.lda = P.n;
          t.aux = c;
          t.a_off = P.ioff + r0;
          t.b_off = P.prow0;
          t.c_off = P.prow0 + r0;
          t.dofs = P.prow0 + r0;
          t.pad0 = stf[c].second - (r0 + sz);  // with pivoting the sum runs to the factor tile's end
          std::vector<Access> ac{{kZKey | gk | c, true}};
          for (int q = st0[I]; q < st0[I + 1]; ++q) ac.push_back({wkey(0, q), false});
          int id = sg.add(t, inpr, wsolve(sz, r0 + sz));
          S.ftile[I].push_back(id);
          S.lastz[c] = id;
          sacc.push_back(ac);
        }
        for (int b = 1; b < P.npb; ++b) {
          const PBlock& B = p.pblocks[P.pb0 + b];
          const Panel& PJ = p.panels[B.J];
          for (int r = st0[B.J]; r < st0[B.J + 1]; ++r) {
            const int r0 = stl[r].first, sz = stl[r].second;
            // the update from a wide panel of the last eighth of the order
            // (the dense top of the tree, whose panels form a chain) is cut
            // into column halves, two tasks into two accumulators: each link
            // of the chain waits for half the product
            const int nh = (P.n >= kSolveKSplitMin && 8 * I >= 7 * nb) ? 2 : 1;
            const int kh = (P.n / 2) & ~1;  // even: the halves' operand columns stay 16-byte aligned
            for (int h = 0; h < nh; ++h) {
              const int k0 = h == 0 ? 0 : kh, k1 = (nh == 1 || h == 1) ? P.n : kh;
              GState::PendF& pf = S.pendf[r];
              if (pf.src.empty()) {
                Task u{};
                u.kind = TK_FUPD | (g << 8);
                u.panel = I;
                u.m = sz;
                u.k = k1 - k0;
                u.lda = P.H;
                u.aux = r;
                u.a_off = P.off + B.prow + r0 + (int64_t)k0 * P.H;  // rows of (L D)_rI in LD, columns k0..
                u.b_off = P.prow0 + k0;                             // rows k0.. of z_I in Z
                u.c_off = PJ.prow0 + r0;
                pf.t = u;
                pf.ac.push_back({0, true});  // the target, set when the slot is known
              }
              pf.pr.insert(pf.pr.end(), S.ftile[I].begin(), S.ftile[I].end());
              for (int c = st0[I]; c < st0[I + 1]; ++c) pf.ac.push_back({kZKey | gk | c, false});
              pf.src.push_back({P.off + B.prow + r0 + (int64_t)k0 * P.H, P.prow0 + k0, k1 - k0, P.H});
              pf.w += tile_work(sz, wn, k1 - k0) / 5.5e5 + (pf.src.size() > 1 ? 3.0 : 0.0);
              if ((int)pf.src.size() >= kMergeSolve) emit_fupd(r);
            }
          }
        }
      }
    };
    auto backward = [&](int g) {
      GState& S = gs[g];
      const int64_t gk = (int64_t)g << 50;
      auto wkey = [&](int slot, int r) { return kWKey | gk | ((int64_t)slot << 40) | r; };
      for (int J = nb - 1; J >= 0; --J) {
        const Panel& PJ = p.panels[J];
        std::vector<int32_t> zpr;
        for (int c = st0[J]; c < st0[J + 1]; ++c) zpr.push_back(S.lastz[c]);
        for (int c = st0[J]; c < st0[J + 1] && J < nfac; ++c) {
          const int r0 = stl[c].first, sz = stl[c].second;
          Task t{};
          t.kind = TK_BTILE | (g << 8);
          t.panel = J;
          t.m = sz;
          t.k = PJ.n - r0;
          t.lda = PJ.n;
          t.aux = c;
          t.a_off = PJ.ioff + r0 + (int64_t)r0 * PJ.n;
          t.b_off = PJ.prow0 + r0;
          t.c_off = PJ.prow0 + r0;
          t.pad0 = r0 - stf[c].first;  // with pivoting the sum starts at the factor tile's first row
          std::vector<Access> ac{{wkey(0, c), true}};
          for (int q = st0[J]; q < st0[J + 1]; ++q) ac.push_back({kZKey | gk | q, false});
          int id = bg.add(t, zpr, wsolve(sz, PJ.n - r0));
          S.btile[J].push_back(id);
          S.lastb[c] = id;
          bacc.push_back(ac);
        }
        for (auto& h : holders[J]) {
          const int I = h.first;
          if (I >= nfac) continue;
          const Panel& P = p.panels[I];
          for (int c = st0[I]; c < st0[I + 1]; ++c) {
            const int r0 = stl[c].first, sz = stl[c].second;
            Task u{};
            u.kind = TK_BUPD | (g << 8);
            u.panel = I;
            u.m = sz;
            u.k = PJ.n;
            u.lda = P.H;
            u.aux = c;
            u.a_off = P.off + h.second + (int64_t)r0 * P.H;
            u.b_off = PJ.prow0;              // rows of x_J in W
            u.c_off = P.prow0 + r0;          // rows of t_c in Z
            std::vector<int32_t> pr2(S.btile[J]);
            pr2.push_back(S.lastz[c]);
            std::vector<Access> ac2{{kZKey | gk | c, true}};
            for (int cc = st0[J]; cc < st0[J + 1]; ++cc) ac2.push_back({wkey(0, cc), false});
            int uid = bg.add(u, pr2, wsolve(sz, PJ.n));
            S.lastz[c] = uid;
            bacc.push_back(ac2);
          }
        }
      }
    };
    for (int g = 0; g < G; ++g) forward(g);
    if (split) {
      // everything of the forward part is done before the backward launch,
      // and x of the blocks left is given
      finalize(sg, p.nworkers, sched, fwd_out);
      if (sg.t.size() <= 40000) fwd_acc = std::move(sacc);
      for (auto& q : gs) {
        std::fill(q.lastz.begin(), q.lastz.end(), -1);
        std::fill(q.lastb.begin(), q.lastb.end(), -1);
      }
    }
    for (int g = 0; g < G; ++g) backward(g);
    if (split) {
      finalize(sgb, p.nworkers, sched, *bwd_out);
      if (sgb.t.size() <= 40000) *bwd_acc = std::move(saccb);
    } else {
      finalize(sg, p.nworkers, sched, fwd_out);
      if (sg.t.size() <= 40000) fwd_acc = std::move(sacc);
    }
  };
  const bool partial = nfac < nb;
  if (partial) {
    gen_solve(1, p.sdag, p.sacc, &p.sdag2, &p.sacc2);
  } else {
    gen_solve(1, p.sdag, p.sacc, nullptr, nullptr);
    if (p.rhs_groups > 1) gen_solve(p.rhs_groups, p.sdagg, p.saccg, nullptr, nullptr);
  }
  // ---- partial elimination: rows of the eliminated blocks, the reduced
  // matrix's K offsets and where its blocks are in panel storage
  if (partial) {
    p.N_elim = 0;
    for (int I = 0; I < nfac; ++I) p.N_elim += p.panels[I].n;
    const int nr = p.nred;
    p.koff_red.assign(nr + p.npair_red + 1, 0);
    for (int i = 0; i < nr; ++i) p.koff_red[i + 1] = p.koff_red[i] + (int64_t)p.n[i] * p.n[i];
    for (int k = 0; k < p.npair_red; ++k)
      p.koff_red[nr + k + 1] = p.koff_red[nr + k] + (int64_t)p.n[p.pairs[k][0]] * p.n[p.pairs[k][1]];
    p.kgather.clear();
    for (int i = 0; i < nr; ++i) {
      const Panel& P = p.panels[p.pos[i]];
      p.kgather.push_back({P.off, p.koff_red[i], P.n, P.n, P.H, 0});
    }
    for (int k = 0; k < p.npair_red; ++k) {
      const int a = p.pairs[k][0], b = p.pairs[k][1];  // K_ab, n_a x n_b
      const int pa = p.pos[a], pb = p.pos[b];
      if (pa > pb) {
        const Panel& P = p.panels[pb];
        p.kgather.push_back({P.off + prow_in[pb][pa], p.koff_red[nr + k], p.n[a], p.n[b], P.H, 0});
      } else {
        const Panel& P = p.panels[pa];
        p.kgather.push_back({P.off + prow_in[pa][pb], p.koff_red[nr + k], p.n[b], p.n[a], P.H, 1});
      }
    }
  }
  *err = 0;
  return "";
}

TaskDag merge_dags(const std::vector<const TaskDag*>& dags, int P) {
  GenDag g;
  for (size_t i = 0; i < dags.size(); ++i) {
    const TaskDag& d = *dags[i];
    const int n = (int)d.tasks.size();
    const int base = (int)g.t.size();
    std::vector<Task> gen(n);
    for (int k = 0; k < n; ++k) gen[d.gen_of[k]] = d.tasks[k];
    for (int q = 0; q < n; ++q) {
      Task t = gen[q];
      t.inst = (int32_t)i;
      std::vector<int32_t> pr;
      for (int x : d.gpreds[q]) pr.push_back(x + base);
      g.t.push_back(t);
      g.preds.push_back(pr);
      g.w.push_back(d.weight_us[q]);
    }
  }
  TaskDag out;
  finalize(g, P, 0, out);
  return out;
}

// Serializability: for every pair of tasks touching one resource where at
// least one writes, the DAG must order them as the sequential elimination
// (the generation order) does.  Reachability by bitsets in generation order.
int64_t check_dag(const TaskDag& dag, const std::vector<std::vector<Access>>& acc) {
  const int n = (int)dag.gpreds.size();
  if ((int)acc.size() != n) return -1;
  const int words = (n + 63) / 64;
  std::vector<uint64_t> reach((size_t)n * words, 0);  // reach[i] = ancestors of i
  for (int i = 0; i < n; ++i) {
    uint64_t* ri = &reach[(size_t)i * words];
    for (int q : dag.gpreds[i]) {
      if (q >= i) return -2;  // generation order must be topological
      const uint64_t* rq = &reach[(size_t)q * words];
      for (int w = 0; w < words; ++w) ri[w] |= rq[w];
      ri[q / 64] |= 1ULL << (q % 64);
    }
  }
  auto before = [&](int a, int b) {  // a is an ancestor of b
    return (reach[(size_t)b * words + a / 64] >> (a % 64)) & 1ULL;
  };
  std::unordered_map<int64_t, std::vector<std::pair<int, bool>>> by_key;
  for (int i = 0; i < n; ++i)
    for (auto& a : acc[i]) by_key[a.key].push_back({i, a.write});
  int64_t bad = 0;
  for (auto& kv : by_key) {
    auto& v = kv.second;
    for (size_t x = 0; x < v.size(); ++x)
      for (size_t y = x + 1; y < v.size(); ++y) {
        if (!v[x].second && !v[y].second) continue;
        int a = v[x].first, b = v[y].first;
        if (a == b) continue;
        int lo = std::min(a, b), hi = std::max(a, b);
        if (!before(lo, hi)) ++bad;
      }
  }
  return bad;
}

}  // namespace d3m
