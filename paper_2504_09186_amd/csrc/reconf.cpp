// Local optimisation of a contraction tree by subtree reconfiguration.
//
// The paper takes its contraction paths from a hyper-optimised external
// search (Evaluation section).  Here a greedy path is refined locally: for a
// node v, the subtree below v is cut at up to kMaxGroups frontier groups
// (leaves or whole subtrees), the optimal contraction order of those groups
// is found by dynamic programming over subsets, and the subtree is replaced
// when that is cheaper.  The index set of any tree node depends only on the
// set of leaves below it (an index stays open while some holder is outside
// or it is an output), so a group is summarised by its open indices and, for
// each, how many of its leaves hold it.  Flops of a pairwise contraction are
// 8 * 2^|indices of both operands|.  Intermediates are kept at most
// 2^cap_bits entries, so a slicing chosen for that cap stays valid.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>

#include "internal.hpp"

namespace mitnc {

namespace {

constexpr int kMaxGroups = 8;

struct Node {
  int left = -1, right = -1, parent = -1;
  std::vector<std::pair<int, int>> open;  // (label, leaves below holding it), sorted by label
  double flops = 0;                       // of the contraction at this node (0 for leaves)
};

struct Ctx {
  const SymNet& sn;
  std::vector<int> total;  // leaves holding each label (removed labels: 0)
  std::vector<char> removed;
  int cap_bits;
};

void merge_open(const Ctx& c, const std::vector<std::pair<int, int>>& a, const std::vector<std::pair<int, int>>& b,
                std::vector<std::pair<int, int>>& out, int& union_size) {
  out.clear();
  union_size = 0;
  size_t i = 0, j = 0;
  while (i < a.size() || j < b.size()) {
    int x, cnt;
    if (j >= b.size() || (i < a.size() && a[i].first < b[j].first)) {
      x = a[i].first;
      cnt = a[i].second;
      ++i;
    } else if (i >= a.size() || b[j].first < a[i].first) {
      x = b[j].first;
      cnt = b[j].second;
      ++j;
    } else {
      x = a[i].first;
      cnt = a[i].second + b[j].second;
      ++i;
      ++j;
    }
    ++union_size;
    if (c.sn.is_out[x] || cnt < c.total[x]) out.push_back({x, cnt});
  }
}

void recompute(const Ctx& c, std::vector<Node>& t, int v) {
  Node& nd = t[v];
  int us;
  merge_open(c, t[nd.left].open, t[nd.right].open, nd.open, us);
  nd.flops = 8.0 * std::ldexp(1.0, us);
}

// Recomputes every internal node bottom-up (post-order from the root).
void recompute_all(const Ctx& c, std::vector<Node>& t, int root) {
  std::vector<int> st{root}, order;
  while (!st.empty()) {
    int v = st.back();
    st.pop_back();
    if (t[v].left < 0) continue;
    order.push_back(v);
    st.push_back(t[v].left);
    st.push_back(t[v].right);
  }
  for (auto it = order.rbegin(); it != order.rend(); ++it) recompute(c, t, *it);
}

// Tries to improve the subtree at v; returns true when it was replaced.
bool reconfigure(const Ctx& c, std::vector<Node>& t, int v) {
  if (t[v].left < 0) return false;
  // frontier expansion: open the most expensive internal group first
  std::vector<int> frontier{t[v].left, t[v].right};
  std::vector<int> inner{v};
  while ((int)frontier.size() < kMaxGroups) {
    int best = -1;
    for (int i = 0; i < (int)frontier.size(); ++i) {
      int g = frontier[i];
      if (t[g].left < 0) continue;
      if (best < 0 || t[g].flops > t[frontier[best]].flops) best = i;
    }
    if (best < 0) break;
    int g = frontier[best];
    frontier.erase(frontier.begin() + best);
    frontier.push_back(t[g].left);
    frontier.push_back(t[g].right);
    inner.push_back(g);
  }
  const int k = (int)frontier.size();
  if (k < 3) return false;
  double current = 0;
  for (int g : inner) current += t[g].flops;
  // local labels
  std::vector<int> labels;
  for (int g : frontier)
    for (auto& [x, n] : t[g].open) labels.push_back(x);
  std::sort(labels.begin(), labels.end());
  labels.erase(std::unique(labels.begin(), labels.end()), labels.end());
  const int nl = (int)labels.size();
  if (nl > 64) return false;
  auto local = [&](int x) { return (int)(std::lower_bound(labels.begin(), labels.end(), x) - labels.begin()); };
  const int NS = 1 << k;
  std::vector<uint64_t> lmask(NS, 0);
  std::vector<std::vector<int>> cnt(NS, std::vector<int>(nl, 0));
  for (int s = 1; s < NS; ++s) {
    int low = __builtin_ctz(s);
    int rest = s & (s - 1);
    std::vector<int>& cs = cnt[s];
    if (rest) cs = cnt[rest];
    for (auto& [x, n] : t[frontier[low]].open) cs[local(x)] += n;
    uint64_t m = 0;
    for (int i = 0; i < nl; ++i) {
      int x = labels[i];
      if (cs[i] > 0 && (c.sn.is_out[x] || cs[i] < c.total[x])) m |= 1ull << i;
    }
    lmask[s] = m;
  }
  const double INF = 1e300;
  std::vector<double> best(NS, INF);
  std::vector<int> split(NS, 0);
  for (int i = 0; i < k; ++i) best[1 << i] = 0;
  for (int s = 1; s < NS; ++s) {
    if (__builtin_popcount(s) < 2) continue;
    if (__builtin_popcountll(lmask[s]) > c.cap_bits && s != NS - 1) continue;  // over the size cap
    const int low = s & -s;
    for (int a = (s - 1) & s; a > 0; a = (a - 1) & s) {
      if (!(a & low)) continue;  // each unordered split once
      const int b = s ^ a;
      if (best[a] >= INF || best[b] >= INF) continue;
      const double f = best[a] + best[b] + 8.0 * std::ldexp(1.0, __builtin_popcountll(lmask[a] | lmask[b]));
      if (f < best[s]) {
        best[s] = f;
        split[s] = a;
      }
    }
  }
  if (!(best[NS - 1] < current * (1.0 - 1e-9))) return false;
  // rebuild: reuse the ids of the replaced inner nodes, v stays on top
  std::vector<int> free_ids(inner.begin() + 1, inner.end());
  std::vector<int> stack_s{NS - 1}, stack_id{v};
  while (!stack_s.empty()) {
    int s = stack_s.back(), id = stack_id.back();
    stack_s.pop_back();
    stack_id.pop_back();
    int a = split[s], b = s ^ a;
    int ids[2];
    int parts[2] = {a, b};
    for (int j = 0; j < 2; ++j) {
      int p = parts[j];
      if (__builtin_popcount(p) == 1) {
        ids[j] = frontier[__builtin_ctz(p)];
      } else {
        ids[j] = free_ids.back();
        free_ids.pop_back();
        stack_s.push_back(p);
        stack_id.push_back(ids[j]);
      }
      t[ids[j]].parent = id;
    }
    t[id].left = ids[0];
    t[id].right = ids[1];
  }
  // recompute the rebuilt nodes bottom-up
  recompute_all(c, t, v);
  return true;
}

}  // namespace

Path optimize_path(const SymNet& sn, const Path& path, const std::vector<char>* removed, int cap_bits, int passes) {
  const int n = (int)sn.leaf.size();
  Ctx c{sn, std::vector<int>(sn.n_labels, 0), std::vector<char>(sn.n_labels, 0), cap_bits};
  if (removed) c.removed = *removed;
  std::vector<Node> t(n + path.size());
  for (int i = 0; i < n; ++i) {
    for (int x : sn.leaf[i])
      if (!c.removed[x]) c.total[x]++;
  }
  for (int i = 0; i < n; ++i)
    for (int x : sn.leaf[i])
      if (!c.removed[x] && (sn.is_out[x] || 1 < c.total[x])) t[i].open.push_back({x, 1});
  for (size_t s = 0; s < path.size(); ++s) {
    int v = n + (int)s;
    t[v].left = path[s].first;
    t[v].right = path[s].second;
    t[path[s].first].parent = v;
    t[path[s].second].parent = v;
  }
  const int root = n + (int)path.size() - 1;
  recompute_all(c, t, root);
  for (int pass = 0; pass < passes; ++pass) {
    std::vector<int> order;
    for (int v = n; v <= root; ++v) order.push_back(v);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return t[a].flops > t[b].flops; });
    int changed = 0;
    for (int v : order) changed += reconfigure(c, t, v);
    if (!changed) break;
  }
  // back to SSA pairs, post-order
  Path out;
  std::vector<int> ssa(t.size(), -1);
  for (int i = 0; i < n; ++i) ssa[i] = i;
  std::vector<std::pair<int, int>> st{{root, 0}};
  while (!st.empty()) {
    auto [v, state] = st.back();
    st.pop_back();
    if (t[v].left < 0) continue;
    if (state == 0) {
      st.push_back({v, 1});
      st.push_back({t[v].right, 0});
      st.push_back({t[v].left, 0});
    } else {
      out.push_back({ssa[t[v].left], ssa[t[v].right]});
      ssa[v] = n + (int)out.size() - 1;
    }
  }
  return out;
}

}  // namespace mitnc
