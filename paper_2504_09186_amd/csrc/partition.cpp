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

// Bisection of the live ids V.  side[i] in {0, 1} for V[i].
struct Bisector {
  const State& S;
  const std::vector<int>& V;
  double ext_weight;
  double imbalance;
  std::mt19937_64& rng;
  int m = 0;
  // local hypergraph
  std::vector<std::vector<int>> vedges;  // per vertex: local edge ids
  std::vector<std::vector<int>> epins;   // per edge: local vertices
  std::vector<double> ew;                // per edge weight

  Bisector(const State& s, const std::vector<int>& v, double ext, double imb, std::mt19937_64& r)
      : S(s), V(v), ext_weight(ext), imbalance(imb), rng(r) {
    m = (int)V.size();
    std::vector<std::vector<int>> in_v;  // label -> local holders
    std::vector<int> lab_edge(S.sn.n_labels, -1);
    vedges.assign(m, {});
    std::vector<int> seen;
    for (int i = 0; i < m; ++i)
      for (int x : S.t[V[i]]) {
        if (lab_edge[x] < 0) {
          lab_edge[x] = (int)epins.size();
          epins.push_back({});
          seen.push_back(x);
        }
        epins[lab_edge[x]].push_back(i);
      }
    // keep edges with >= 2 pins in V
    std::vector<int> remap(epins.size(), -1);
    std::vector<std::vector<int>> pins2;
    for (size_t e = 0; e < epins.size(); ++e) {
      if (epins[e].size() < 2) continue;
      const int x = seen[e];
      const bool internal = !S.sn.is_out[x] && S.count[x] == (int)epins[e].size();
      remap[e] = (int)pins2.size();
      pins2.push_back(epins[e]);
      ew.push_back(internal ? 1.0 : ext_weight);
    }
    epins.swap(pins2);
    for (size_t e = 0; e < epins.size(); ++e)
      for (int v : epins[e]) vedges[v].push_back((int)e);
  }

  double cut_of(const std::vector<int>& side) const {
    double c = 0;
    for (size_t e = 0; e < epins.size(); ++e) {
      int n1 = 0;
      for (int v : epins[e]) n1 += side[v];
      if (n1 > 0 && n1 < (int)epins[e].size()) c += ew[e];
    }
    return c;
  }

  // Greedy growth of side 1 from a random vertex up to `target` vertices.
  void grow(std::vector<int>& side, int target) {
    side.assign(m, 0);
    std::vector<double> conn(m, 0.0);  // weight of edges into the grown part
    std::uniform_int_distribution<int> pick(0, m - 1);
    int seed = pick(rng);
    int size = 0;
    std::uniform_real_distribution<double> jit(0.0, 1e-3);
    auto add = [&](int v) {
      side[v] = 1;
      ++size;
      for (int e : vedges[v])
        for (int u : epins[e])
          if (!side[u]) conn[u] += ew[e];
    };
    add(seed);
    while (size < target) {
      int best = -1;
      double bv = -1e300;
      for (int v = 0; v < m; ++v) {
        if (side[v]) continue;
        // prefer vertices tied to the part, with few ties elsewhere
        double other = 0;
        for (int e : vedges[v]) other += ew[e];
        const double g = 2 * conn[v] - other + jit(rng);
        if (g > bv) {
          bv = g;
          best = v;
        }
      }
      add(best);
    }
  }

  // Fiduccia-Mattheyses passes; side sizes kept within [lo, hi].
  void refine(std::vector<int>& side, int lo, int hi) {
    std::vector<std::array<int, 2>> cnt(epins.size());
    auto recount = [&]() {
      for (size_t e = 0; e < epins.size(); ++e) {
        cnt[e] = {0, 0};
        for (int v : epins[e]) cnt[e][side[v]]++;
      }
    };
    auto gain = [&](int v) {
      const int s = side[v];
      double g = 0;
      for (int e : vedges[v]) {
        if (cnt[e][s] == 1 && cnt[e][1 - s] > 0) g += ew[e];
        else if (cnt[e][1 - s] == 0 && cnt[e][s] > 1) g -= ew[e];
      }
      return g;
    };
    for (int pass = 0; pass < 8; ++pass) {
      recount();
      int n1 = 0;
      for (int v = 0; v < m; ++v) n1 += side[v];
      std::vector<double> g(m);
      for (int v = 0; v < m; ++v) g[v] = gain(v);
      std::vector<char> locked(m, 0);
      std::vector<int> moves;
      double cum = 0, best_cum = 0;
      size_t best_len = 0;
      for (int step = 0; step < m; ++step) {
        int bv = -1;
        double bg = -1e300;
        for (int v = 0; v < m; ++v) {
          if (locked[v]) continue;
          const int n1_after = n1 + (side[v] ? -1 : 1);
          if (n1_after < lo || n1_after > hi) continue;
          if (g[v] > bg) {
            bg = g[v];
            bv = v;
          }
        }
        if (bv < 0) break;
        // move bv
        const int s = side[bv];
        for (int e : vedges[bv]) {
          cnt[e][s]--;
          cnt[e][1 - s]++;
        }
        side[bv] = 1 - s;
        n1 += s ? -1 : 1;
        locked[bv] = 1;
        cum += bg;
        moves.push_back(bv);
        for (int e : vedges[bv])
          for (int u : epins[e])
            if (!locked[u]) g[u] = gain(u);
        if (cum > best_cum + 1e-12) {
          best_cum = cum;
          best_len = moves.size();
        }
      }
      // roll back past the best prefix
      for (size_t k = moves.size(); k > best_len; --k) side[moves[k - 1]] ^= 1;
      if (best_len == 0) break;
    }
  }

  std::vector<int> run(int starts) {
    std::vector<int> best;
    double best_cut = 0;
    const double half = m / 2.0;
    const int lo = std::max(1, (int)std::floor(half * (1.0 - imbalance)));
    const int hi = std::min(m - 1, (int)std::ceil(half * (1.0 + imbalance)));
    std::uniform_int_distribution<int> tg(lo, hi);
    for (int st = 0; st < starts; ++st) {
      std::vector<int> side;
      grow(side, tg(rng));
      refine(side, lo, hi);
      const double c = cut_of(side);
      if (best.empty() || c < best_cut) {
        best = side;
        best_cut = c;
      }
    }
    return best;
  }
};

int build(State& S, const std::vector<int>& V, const PartitionParams& prm, std::mt19937_64& rng) {
  if (V.size() == 1) return V[0];
  if ((int)V.size() <= prm.cutoff) return greedy_part(S, V);
  Bisector bs(S, V, prm.ext_weight, prm.imbalance, rng);
  std::vector<int> side = bs.run(prm.starts);
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
