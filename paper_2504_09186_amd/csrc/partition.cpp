// Contraction paths by recursive bisection of the network.
//
// The paper takes its contraction paths from an external hyper-optimised
// search (Evaluation section); the cost it cares about is the size of the
// intermediates (memory, hence slicing, Sec. III-A) and the flops of the
// pairwise contractions (Sec. II-A).  This search builds the contraction
// tree top-down instead of greedily bottom-up:
//
//  1. Free merges.  A tensor whose contraction with a neighbour yields no
//     more indices than the larger of the two has (single-qubit gates and
//     the |0> / projector vectors absorbed into two-qubit gates) is merged
//     first, smallest first; each merge is one contraction step.
//  2. Bisection.  The remaining tensors are split in two parts that share
//     few indices, recursively; a split is a tree node whose two children
//     are contracted last.  Indices held only inside the part being split
//     (and not requested outputs) cost weight 1 when cut (they enlarge
//     this node's contraction); indices also held outside cost `ext_weight`
//     (they enlarge the children).  A split starts from a part grown
//     greedily around a random tensor and is refined by Fiduccia-Mattheyses
//     passes (single moves by largest gain, best prefix kept), several
//     starts, under the balance bound |part| within (1 +- imbalance) / 2.
//  3. Parts of at most `cutoff` tensors are contracted greedily (lowest
//     size(out) - size(a) - size(b) first).
//
// The index set of any intermediate depends only on the leaves below it: an
// index stays while a leaf outside holds it or it is an output.  The search
// keeps a count of live tensors per index to evaluate that on the fly.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <random>

#include "internal.hpp"

namespace mitnc {

namespace {

struct State {
  const SymNet& sn;
  const std::vector<char>& removed;
  std::vector<std::vector<int>> t;  // labels of every SSA id (sorted)
  std::vector<int> count;           // live tensors holding each label
  Path path;
  int n_leaves;
};

// Labels of the contraction of ids a and b (does not modify the state).
void merged_labels(const State& S, int a, int b, std::vector<int>& c) {
  c.clear();
  const auto& A = S.t[a];
  const auto& B = S.t[b];
  size_t i = 0, j = 0;
  while (i < A.size() || j < B.size()) {
    int x, held;
    if (j >= B.size() || (i < A.size() && A[i] < B[j])) {
      x = A[i++];
      held = 1;
    } else if (i >= A.size() || B[j] < A[i]) {
      x = B[j++];
      held = 1;
    } else {
      x = A[i];
      ++i;
      ++j;
      held = 2;
    }
    if (S.count[x] - held > 0 || S.sn.is_out[x]) c.push_back(x);
  }
}

int contract(State& S, int a, int b) {
  std::vector<int> c;
  merged_labels(S, a, b, c);
  for (int x : S.t[a]) S.count[x]--;
  for (int x : S.t[b]) S.count[x]--;
  for (int x : c) S.count[x]++;
  const int id = (int)S.t.size();
  S.t.push_back(std::move(c));
  std::vector<int>().swap(S.t[a]);
  std::vector<int>().swap(S.t[b]);
  S.path.push_back({a, b});
  return id;
}

// Phase 1: merges that do not grow the larger tensor.  Returns live ids.
std::vector<int> free_merges(State& S) {
  std::vector<int> live(S.n_leaves);
  std::iota(live.begin(), live.end(), 0);
  std::vector<char> alive(S.n_leaves, 1);
  std::vector<std::vector<int>> holders(S.sn.n_labels);
  for (int i = 0; i < S.n_leaves; ++i)
    for (int x : S.t[i]) holders[x].push_back(i);
  std::vector<int> c;
  bool changed = true;
  while (changed) {
    changed = false;
    std::vector<int> order;
    for (int v : live)
      if (alive[v]) order.push_back(v);
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return S.t[u].size() < S.t[v].size(); });
    for (int v : order) {
      if (!alive[v]) continue;
      int best = -1;
      size_t best_size = 0;
      for (int x : S.t[v]) {
        for (int u : holders[x]) {
          if (u == v || !alive[u]) continue;
          merged_labels(S, v, u, c);
          const size_t lim = std::max(S.t[v].size(), S.t[u].size());
          if (c.size() <= lim && (best < 0 || c.size() < best_size)) {
            best = u;
            best_size = c.size();
          }
        }
      }
      if (best < 0) continue;
      const int a = std::min(v, best), b = std::max(v, best);
      const int id = contract(S, a, b);
      alive[a] = alive[b] = 0;
      alive.push_back(1);
      live.push_back(id);
      for (int x : S.t[id]) holders[x].push_back(id);
      changed = true;
    }
    for (auto& h : holders)
      h.erase(std::remove_if(h.begin(), h.end(), [&](int k) { return !alive[k]; }), h.end());
  }
  std::vector<int> out;
  for (int v : live)
    if (alive[v]) out.push_back(v);
  return out;
}

// Greedy contraction of the ids in V (all live); returns the result id.
int greedy_part(State& S, std::vector<int> V) {
  std::vector<int> c;
  while (V.size() > 1) {
    double best = 0;
    int bi = -1, bj = -1;
    for (size_t i = 0; i < V.size(); ++i)
      for (size_t j = i + 1; j < V.size(); ++j) {
        const auto& A = S.t[V[i]];
        const auto& B = S.t[V[j]];
        bool share = false;
        for (size_t p = 0, q = 0; p < A.size() && q < B.size();) {
          if (A[p] == B[q]) {
            share = true;
            break;
          }
          if (A[p] < B[q]) ++p;
          else ++q;
        }
        merged_labels(S, V[i], V[j], c);
        double cost = std::ldexp(1.0, (int)c.size()) - std::ldexp(1.0, (int)A.size()) -
                      std::ldexp(1.0, (int)B.size());
        if (!share) cost += 1e300;  // outer products only when nothing else is left
        if (bi < 0 || cost < best) {
          best = cost;
          bi = (int)i;
          bj = (int)j;
        }
      }
    const int a = V[bi], b = V[bj];
    const int id = contract(S, std::min(a, b), std::max(a, b));
    V.erase(V.begin() + bj);
    V.erase(V.begin() + bi);
    V.push_back(id);
  }
  return V[0];
}

// Hypergraph of one bisection: vertices with weights (tensors merged by
// coarsening), nets with weights (indices).
struct Graph {
  int m = 0;
  std::vector<int> vw;                   // vertex weights
  std::vector<std::vector<int>> vedges;  // per vertex: incident nets
  std::vector<std::vector<int>> epins;   // per net: vertices (distinct)
  std::vector<double> ew;                // net weights
  int total_weight() const { return std::accumulate(vw.begin(), vw.end(), 0); }
};

Graph local_graph(const State& S, const std::vector<int>& V, double ext_weight) {
  Graph g;
  g.m = (int)V.size();
  g.vw.assign(g.m, 1);
  g.vedges.assign(g.m, {});
  std::vector<int> lab_net(S.sn.n_labels, -1), net_lab;
  std::vector<std::vector<int>> pins;
  for (int i = 0; i < g.m; ++i)
    for (int x : S.t[V[i]]) {
      if (lab_net[x] < 0) {
        lab_net[x] = (int)pins.size();
        pins.push_back({});
        net_lab.push_back(x);
      }
      pins[lab_net[x]].push_back(i);
    }
  for (size_t e = 0; e < pins.size(); ++e) {
    if (pins[e].size() < 2) continue;  // a net on one vertex is never cut
    const int x = net_lab[e];
    const bool internal = !S.sn.is_out[x] && S.count[x] == (int)pins[e].size();
    g.epins.push_back(pins[e]);
    g.ew.push_back(internal ? 1.0 : ext_weight);
  }
  for (size_t e = 0; e < g.epins.size(); ++e)
    for (int v : g.epins[e]) g.vedges[v].push_back((int)e);
  return g;
}

// Heavy-net matching: each vertex pairs with the unmatched neighbour it
// shares the most net weight with (per unit of combined vertex weight).
// map[v] = coarse vertex.  Returns the coarse graph.
Graph coarsen(const Graph& g, std::vector<int>& map, std::mt19937_64& rng, int max_vw) {
  std::vector<int> order(g.m);
  std::iota(order.begin(), order.end(), 0);
  std::shuffle(order.begin(), order.end(), rng);
  std::vector<int> match(g.m, -1);
  std::vector<double> conn(g.m, 0.0);
  std::vector<int> touched;
  for (int v : order) {
    if (match[v] >= 0) continue;
    touched.clear();
    for (int e : g.vedges[v]) {
      const double w = g.ew[e] / (double)(g.epins[e].size() - 1);
      for (int u : g.epins[e])
        if (u != v && match[u] < 0) {
          if (conn[u] == 0.0) touched.push_back(u);
          conn[u] += w;
        }
    }
    int best = -1;
    double bv = 0;
    for (int u : touched) {
      if (g.vw[u] + g.vw[v] <= max_vw) {
        const double sc = conn[u] / (double)(g.vw[u] + g.vw[v]);
        if (sc > bv) {
          bv = sc;
          best = u;
        }
      }
      conn[u] = 0.0;
    }
    match[v] = best >= 0 ? best : v;
    if (best >= 0) match[best] = v;
  }
  Graph c;
  map.assign(g.m, -1);
  for (int v = 0; v < g.m; ++v) {
    if (map[v] >= 0) continue;
    map[v] = c.m;
    if (match[v] != v) map[match[v]] = c.m;
    c.vw.push_back(g.vw[v] + (match[v] != v ? g.vw[match[v]] : 0));
    ++c.m;
  }
  c.vedges.assign(c.m, {});
  std::vector<int> stamp(c.m, -1);
  for (size_t e = 0; e < g.epins.size(); ++e) {
    std::vector<int> p;
    for (int v : g.epins[e]) {
      const int cv = map[v];
      if (stamp[cv] != (int)e) {
        stamp[cv] = (int)e;
        p.push_back(cv);
      }
    }
    if (p.size() < 2) continue;
    c.epins.push_back(std::move(p));
    c.ew.push_back(g.ew[e]);
  }
  for (size_t e = 0; e < c.epins.size(); ++e)
    for (int v : c.epins[e]) c.vedges[v].push_back((int)e);
  return c;
}

double cut_of(const Graph& g, const std::vector<int>& side) {
  double c = 0;
  for (size_t e = 0; e < g.epins.size(); ++e) {
    int n1 = 0;
    for (int v : g.epins[e]) n1 += side[v];
    if (n1 > 0 && n1 < (int)g.epins[e].size()) c += g.ew[e];
  }
  return c;
}

// Fiduccia-Mattheyses passes; the weight of side 1 stays within [lo, hi].
void fm_refine(const Graph& g, std::vector<int>& side, int lo, int hi, int max_passes) {
  const int m = g.m;
  std::vector<std::array<int, 2>> cnt(g.epins.size());
  auto gain = [&](int v) {
    const int s = side[v];
    double r = 0;
    for (int e : g.vedges[v]) {
      if (cnt[e][s] == 1 && cnt[e][1 - s] > 0) r += g.ew[e];
      else if (cnt[e][1 - s] == 0 && cnt[e][s] > 1) r -= g.ew[e];
    }
    return r;
  };
  for (int pass = 0; pass < max_passes; ++pass) {
    for (size_t e = 0; e < g.epins.size(); ++e) {
      cnt[e] = {0, 0};
      for (int v : g.epins[e]) cnt[e][side[v]]++;
    }
    int w1 = 0;
    for (int v = 0; v < m; ++v) w1 += side[v] * g.vw[v];
    std::vector<double> gv(m);
    for (int v = 0; v < m; ++v) gv[v] = gain(v);
    std::vector<char> locked(m, 0);
    std::vector<int> moves;
    double cum = 0, best_cum = 0;
    size_t best_len = 0;
    for (int step = 0; step < m; ++step) {
      int bv = -1;
      double bg = -1e300;
      for (int v = 0; v < m; ++v) {
        if (locked[v]) continue;
        const int w_after = w1 + (side[v] ? -g.vw[v] : g.vw[v]);
        if (w_after < lo || w_after > hi) continue;
        if (gv[v] > bg) {
          bg = gv[v];
          bv = v;
        }
      }
      if (bv < 0) break;
      const int s = side[bv];
      for (int e : g.vedges[bv]) {
        cnt[e][s]--;
        cnt[e][1 - s]++;
      }
      side[bv] = 1 - s;
      w1 += s ? -g.vw[bv] : g.vw[bv];
      locked[bv] = 1;
      cum += bg;
      moves.push_back(bv);
      for (int e : g.vedges[bv])
        for (int u : g.epins[e])
          if (!locked[u]) gv[u] = gain(u);
      if (cum > best_cum + 1e-12) {
        best_cum = cum;
        best_len = moves.size();
      }
    }
    for (size_t k = moves.size(); k > best_len; --k) side[moves[k - 1]] ^= 1;
    if (best_len == 0) break;
  }
}

// Greedy growth of side 1 from a random vertex up to weight `target`.
void grow(const Graph& g, std::vector<int>& side, int target, std::mt19937_64& rng) {
  side.assign(g.m, 0);
  std::vector<double> conn(g.m, 0.0), deg(g.m, 0.0);
  for (int v = 0; v < g.m; ++v)
    for (int e : g.vedges[v]) deg[v] += g.ew[e];
  std::uniform_real_distribution<double> jit(0.0, 1e-3);
  int w = 0;
  auto add = [&](int v) {
    side[v] = 1;
    w += g.vw[v];
    for (int e : g.vedges[v])
      for (int u : g.epins[e])
        if (!side[u]) conn[u] += g.ew[e];
  };
  add(std::uniform_int_distribution<int>(0, g.m - 1)(rng));
  while (w < target) {
    int best = -1;
    double bv = -1e300;
    for (int v = 0; v < g.m; ++v) {
      if (side[v]) continue;
      const double sc = 2 * conn[v] - deg[v] + jit(rng);
      if (sc > bv) {
        bv = sc;
        best = v;
      }
    }
    if (best < 0) break;
    add(best);
  }
}

// Multilevel bisection: coarsen to at most `coarse_m` vertices, several
// grown and refined starts there, then project back refining each level.
std::vector<int> bisect(const Graph& g0, double imbalance, int starts, std::mt19937_64& rng) {
  const int W = g0.total_weight();
  const double half = W / 2.0;
  const int lo = std::max(1, (int)std::floor(half * (1.0 - imbalance)));
  const int hi = std::min(W - 1, (int)std::ceil(half * (1.0 + imbalance)));
  std::vector<Graph> levels{g0};
  std::vector<std::vector<int>> maps;
  const int coarse_m = 40;
  while (levels.back().m > coarse_m) {
    std::vector<int> map;
    Graph c = coarsen(levels.back(), map, rng, std::max(2, W / 8));
    if (c.m > 0.9 * levels.back().m) break;  // matching stalled
    maps.push_back(std::move(map));
    levels.push_back(std::move(c));
  }
  const Graph& gc = levels.back();
  std::vector<int> best;
  double best_cut = 0;
  std::uniform_int_distribution<int> tg(lo, hi);
  for (int st = 0; st < starts; ++st) {
    std::vector<int> side;
    grow(gc, side, tg(rng), rng);
    fm_refine(gc, side, lo, hi, 8);
    int w1 = 0;
    for (int v = 0; v < gc.m; ++v) w1 += side[v] * gc.vw[v];
    if (w1 < lo || w1 > hi) continue;
    const double c = cut_of(gc, side);
    if (best.empty() || c < best_cut) {
      best = side;
      best_cut = c;
    }
  }
  if (best.empty()) {  // no balanced start at the coarsest level: grow on the finest
    grow(g0, best, (lo + hi) / 2, rng);
    fm_refine(g0, best, lo, hi, 8);
    return best;
  }
  for (int L = (int)levels.size() - 2; L >= 0; --L) {
    std::vector<int> fine(levels[L].m);
    for (int v = 0; v < levels[L].m; ++v) fine[v] = best[maps[L][v]];
    best.swap(fine);
    fm_refine(levels[L], best, lo, hi, 8);
  }
  return best;
}

int build(State& S, const std::vector<int>& V, const PartitionParams& prm, std::mt19937_64& rng) {
  if (V.size() == 1) return V[0];
  if ((int)V.size() <= prm.cutoff) return greedy_part(S, V);
  const Graph g = local_graph(S, V, prm.ext_weight);
  std::vector<int> side = bisect(g, prm.imbalance, prm.starts, rng);
  std::vector<int> V0, V1;
  for (size_t i = 0; i < V.size(); ++i) (side[i] ? V1 : V0).push_back(V[i]);
  if (V0.empty() || V1.empty()) return greedy_part(S, V);
  const int a = build(S, V0, prm, rng);
  const int b = build(S, V1, prm, rng);
  return contract(S, std::min(a, b), std::max(a, b));
}

}  // namespace

Path partition_path(const SymNet& sn, const std::vector<char>& removed, const PartitionParams& prm, uint64_t seed) {
  State S{sn, removed, {}, std::vector<int>(sn.n_labels, 0), {}, (int)sn.leaf.size()};
  S.t.resize(S.n_leaves);
  for (int i = 0; i < S.n_leaves; ++i) {
    for (int x : sn.leaf[i])
      if (!removed[x]) S.t[i].push_back(x);
    for (int x : S.t[i]) S.count[x]++;
  }
  std::mt19937_64 rng(seed);
  std::vector<int> live = free_merges(S);
  build(S, live, prm, rng);
  // the SSA ids of `contract` follow emission order, which is the path order
  return S.path;
}

}  // namespace mitnc
