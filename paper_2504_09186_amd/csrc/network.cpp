// Circuit -> tensor network, symbolic contraction, greedy path and slicing.
//
// Paper, Sec. II-A: the circuit is a tensor network; a contraction removes the
// shared edges of two tensors.  Paper, Sec. III-A: slicing fixes indices so
// that the largest intermediate fits memory, at the price of recomputation;
// the index overhead of Eq. (1) measures that price per index.  The paper
// takes its paths from an external hyper-optimised search; here a randomised
// greedy search stands in for it.
#include <algorithm>
#include <cmath>
#include <queue>
#include <random>
#include <tuple>

#include "internal.hpp"

namespace mitnc {

void fail(int32_t code, const std::string& msg) { throw Error{code, msg}; }

SymNet make_symnet(const std::vector<Leaf>& leaves, const std::vector<int64_t>& output) {
  SymNet sn;
  auto get = [&](int64_t id) {
    auto it = sn.dense.find(id);
    if (it != sn.dense.end()) return it->second;
    int d = sn.n_labels++;
    sn.dense[id] = d;
    sn.label_id.push_back(id);
    return d;
  };
  for (const Leaf& l : leaves) {
    std::vector<int> v;
    for (int64_t id : l.labels) v.push_back(get(id));
    std::sort(v.begin(), v.end());
    sn.leaf.push_back(v);
  }
  for (int64_t id : output) get(id);
  sn.is_out.assign(sn.n_labels, 0);
  for (int64_t id : output) sn.is_out[sn.dense[id]] = 1;
  std::vector<int> count(sn.n_labels, 0);
  for (auto& v : sn.leaf)
    for (int x : v) count[x]++;
  sn.closed.assign(sn.n_labels, 0);
  for (int x = 0; x < sn.n_labels; ++x)
    sn.closed[x] = (count[x] == 2 && !sn.is_out[x] && sn.label_id[x] >= 0);
  return sn;
}

// Output labels of contracting a and b: a label survives if another live
// tensor still holds it or it is an output label.
static void out_labels(const std::vector<int>& a, const std::vector<int>& b, const std::vector<int>& count,
                       const std::vector<char>& is_out, std::vector<int>& c, int& kbits) {
  c.clear();
  kbits = 0;
  size_t i = 0, j = 0;
  while (i < a.size() || j < b.size()) {
    int x;
    int held;
    if (j >= b.size() || (i < a.size() && a[i] < b[j])) {
      x = a[i++];
      held = 1;
    } else if (i >= a.size() || b[j] < a[i]) {
      x = b[j++];
      held = 1;
    } else {
      x = a[i];
      ++i;
      ++j;
      held = 2;
    }
    if (count[x] - held > 0 || is_out[x]) {
      c.push_back(x);
    } else if (held == 2) {
      kbits += 1;
    }
    // a label held once, not output and not elsewhere would be summed alone;
    // circuit networks have none.
  }
}

std::vector<SymStep> sym_run(const SymNet& sn, const Path& path, const std::vector<char>& sliced) {
  size_t n = sn.leaf.size();
  std::vector<std::vector<int>> t(n + path.size());
  std::vector<int> count(sn.n_labels, 0);
  for (size_t i = 0; i < n; ++i) {
    for (int x : sn.leaf[i])
      if (!sliced[x]) t[i].push_back(x);
    for (int x : t[i]) count[x]++;
  }
  std::vector<SymStep> out;
  out.reserve(path.size());
  for (size_t s = 0; s < path.size(); ++s) {
    SymStep st;
    st.a = path[s].first;
    st.b = path[s].second;
    out_labels(t[st.a], t[st.b], count, sn.is_out, st.c, st.k_bits);
    for (int x : t[st.a]) count[x]--;
    for (int x : t[st.b]) count[x]--;
    for (int x : st.c) count[x]++;
    st.c_bits = (int)st.c.size();
    st.flops = 8.0 * std::ldexp(1.0, st.c_bits + st.k_bits);
    t[n + s] = st.c;
    std::vector<int>().swap(t[st.a]);
    std::vector<int>().swap(t[st.b]);
    out.push_back(std::move(st));
  }
  return out;
}

double sym_total_flops(const std::vector<SymStep>& st) {
  double f = 0;
  for (auto& s : st) f += s.flops;
  return f;
}

int sym_max_bits(const SymNet& sn, const std::vector<SymStep>& st, const std::vector<char>& sliced) {
  int m = 0;
  for (auto& v : sn.leaf) {
    int r = 0;
    for (int x : v) r += !sliced[x];
    m = std::max(m, r);
  }
  for (auto& s : st) m = std::max(m, s.c_bits);
  return m;
}

void validate_path(int n_leaves, const Path& path) {
  if ((int)path.size() != n_leaves - 1) fail(MITNC_PATH_INVALID, "path must have n_leaves - 1 steps");
  std::vector<char> alive(n_leaves + path.size(), 0);
  for (int i = 0; i < n_leaves; ++i) alive[i] = 1;
  for (size_t s = 0; s < path.size(); ++s) {
    int a = path[s].first, b = path[s].second;
    if (a < 0 || b < 0 || a == b || a >= (int)(n_leaves + s) || b >= (int)(n_leaves + s) || !alive[a] ||
        !alive[b])
      fail(MITNC_PATH_INVALID, "path step " + std::to_string(s) + " uses an unavailable tensor");
    alive[a] = alive[b] = 0;
    alive[n_leaves + s] = 1;
  }
}

// Randomised greedy: repeatedly contract the connected pair with the lowest
// cost size(out) - alpha * (size(a) + size(b)); with temperature > 0 every
// cost is perturbed by temperature * |cost| * Gumbel noise.  Labels marked in
// `removed` (sliced indices) are ignored.
Path greedy_path(const SymNet& sn, double alpha, double temperature, uint64_t seed,
                 const std::vector<char>* removed) {
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> uni(1e-12, 1.0 - 1e-12);
  size_t n = sn.leaf.size();
  std::vector<std::vector<int>> t(2 * n);
  std::vector<char> alive(2 * n, 0);
  std::vector<int> count(sn.n_labels, 0);
  std::vector<std::vector<int>> holders(sn.n_labels);
  for (size_t i = 0; i < n; ++i) {
    for (int x : sn.leaf[i])
      if (!removed || !(*removed)[x]) t[i].push_back(x);
    alive[i] = 1;
    for (int x : t[i]) {
      count[x]++;
      holders[x].push_back((int)i);
    }
  }
  typedef std::tuple<double, int, int> Item;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  std::vector<int> tmp;
  auto push = [&](int i, int j) {
    if (i > j) std::swap(i, j);
    int kb;
    out_labels(t[i], t[j], count, sn.is_out, tmp, kb);
    double cost = std::ldexp(1.0, (int)tmp.size()) -
                  alpha * (std::ldexp(1.0, (int)t[i].size()) + std::ldexp(1.0, (int)t[j].size()));
    if (temperature > 0) cost += temperature * std::fabs(cost) * (-std::log(-std::log(uni(rng))));
    heap.emplace(cost, i, j);
  };
  for (int x = 0; x < sn.n_labels; ++x) {
    auto& h = holders[x];
    for (size_t a = 0; a < h.size(); ++a)
      for (size_t b = a + 1; b < h.size(); ++b) push(h[a], h[b]);
  }
  Path path;
  size_t live = n;
  int nxt = (int)n;
  while (live > 1) {
    int i = -1, j = -1;
    while (!heap.empty()) {
      auto [c, a, b] = heap.top();
      heap.pop();
      (void)c;
      if (alive[a] && alive[b]) {
        i = a;
        j = b;
        break;
      }
    }
    if (i < 0) {  // disconnected: join the two smallest live tensors
      std::vector<std::pair<size_t, int>> ls;
      for (int k = 0; k < nxt; ++k)
        if (alive[k]) ls.push_back({t[k].size(), k});
      std::sort(ls.begin(), ls.end());
      i = std::min(ls[0].second, ls[1].second);
      j = std::max(ls[0].second, ls[1].second);
    }
    std::vector<int> c;
    int kb;
    out_labels(t[i], t[j], count, sn.is_out, c, kb);
    for (int x : t[i]) count[x]--;
    for (int x : t[j]) count[x]--;
    alive[i] = alive[j] = 0;
    t[nxt] = c;
    alive[nxt] = 1;
    std::vector<int> nb;
    for (int x : c) {
      count[x]++;
      auto& h = holders[x];
      h.erase(std::remove_if(h.begin(), h.end(), [&](int k) { return !alive[k]; }), h.end());
      for (int k : h) nb.push_back(k);
      h.push_back(nxt);
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    for (int k : nb) push(k, nxt);
    path.push_back({i, j});
    ++nxt;
    --live;
  }
  return path;
}

// Greedy slicing: while the largest intermediate exceeds 2^cap (or fewer than
// min_sliced indices are sliced), slice the closed index, among those of the
// largest intermediates, that gives the smallest (largest intermediate,
// per-subtask flops, label id).
std::vector<int> greedy_slices(const SymNet& sn, const Path& path, int cap, int min_sliced, int max_sliced,
                               bool* ok) {
  std::vector<char> sl(sn.n_labels, 0);
  std::vector<int> chosen;
  *ok = false;
  while ((int)chosen.size() <= max_sliced) {
    auto st = sym_run(sn, path, sl);
    int mx = sym_max_bits(sn, st, sl);
    if (mx <= cap && (int)chosen.size() >= min_sliced) {
      *ok = true;
      break;
    }
    if ((int)chosen.size() == max_sliced) break;
    std::vector<char> cand(sn.n_labels, 0);
    for (auto& s : st)
      if (s.c_bits == mx)
        for (int x : s.c)
          if (sn.closed[x] && !sl[x]) cand[x] = 1;
    bool any = false;
    for (int x = 0; x < sn.n_labels; ++x) any |= cand[x];
    if (!any)
      for (int x = 0; x < sn.n_labels; ++x) cand[x] = sn.closed[x] && !sl[x];
    int best = -1;
    std::pair<int, double> bkey{1 << 30, 0.0};
    for (int x = 0; x < sn.n_labels; ++x) {
      if (!cand[x]) continue;
      sl[x] = 1;
      auto s2 = sym_run(sn, path, sl);
      std::pair<int, double> key{sym_max_bits(sn, s2, sl), sym_total_flops(s2)};
      sl[x] = 0;
      if (best < 0 || key < bkey || (key == bkey && sn.label_id[x] < sn.label_id[best])) {
        best = x;
        bkey = key;
      }
    }
    if (best < 0) break;
    sl[best] = 1;
    chosen.push_back(best);
  }
  return chosen;
}

// Slicing interleaved with subtree reconfiguration: slices greedily (the
// rule of greedy_slices) one index at a time, and after every `every`
// indices re-optimises the tree for the sliced network under the current
// largest intermediate, so later choices see the improved tree.  Returns the
// sliced indices; `path` is updated in place.
std::vector<int> slice_reconf(const SymNet& sn, Path& path, const std::vector<int>& fixed, int cap, int min_sliced,
                              int max_sliced, int every, bool* ok) {
  std::vector<char> sl(sn.n_labels, 0);
  for (int x : fixed) sl[x] = 1;
  std::vector<int> chosen;
  *ok = false;
  SymNet sub = sn;
  for (int x : fixed) sub.closed[x] = 0;
  while (true) {
    auto st = sym_run(sn, path, sl);
    int mx = sym_max_bits(sn, st, sl);
    if (mx <= cap && (int)(chosen.size() + fixed.size()) >= min_sliced) {
      *ok = true;
      break;
    }
    if ((int)(chosen.size() + fixed.size()) >= max_sliced) break;
    std::vector<char> cand(sn.n_labels, 0);
    for (auto& s : st)
      if (s.c_bits == mx)
        for (int x : s.c)
          if (sub.closed[x] && !sl[x]) cand[x] = 1;
    bool any = false;
    for (int x = 0; x < sn.n_labels; ++x) any |= cand[x];
    if (!any)
      for (int x = 0; x < sn.n_labels; ++x) cand[x] = sub.closed[x] && !sl[x];
    int best = -1;
    std::pair<int, double> bkey{1 << 30, 0.0};
    for (int x = 0; x < sn.n_labels; ++x) {
      if (!cand[x]) continue;
      sl[x] = 1;
      auto s2 = sym_run(sn, path, sl);
      std::pair<int, double> key{sym_max_bits(sn, s2, sl), sym_total_flops(s2)};
      sl[x] = 0;
      if (best < 0 || key < bkey || (key == bkey && sn.label_id[x] < sn.label_id[best])) {
        best = x;
        bkey = key;
      }
    }
    if (best < 0) break;
    sl[best] = 1;
    chosen.push_back(best);
    if (every > 0 && chosen.size() % every == 0) {
      const int width = sym_max_bits(sn, sym_run(sn, path, sl), sl);
      path = optimize_path(sn, path, &sl, std::max(width, cap), 2);
    }
  }
  return chosen;
}

// Flops of all 2^S slices, run in slice-id order with shared-prefix reuse
// (Sec. III-B): a step whose subtree holds sliced indices with lowest
// slice-id bit b is recomputed 2^(S - b) times, a step with none once.
// `ordered` lists the sliced indices outer -> inner (the last is bit 0).
// With merge_bits > 0 the innermost merge_bits bits (within the window) may
// also be merged after their lifetime ends (post-lifetime reuse; the rule of
// merge_sets), which the counts then include.  launch_cost (flops) is added
// for every step computation, a stand-in for the fixed cost of a kernel
// launch.
double reuse_total_flops(const SymNet& sn, const Path& path, const std::vector<int>& ordered, int window_bits,
                         int merge_bits, double launch_cost) {
  const int S = (int)ordered.size();
  std::vector<char> sl(sn.n_labels, 0);
  std::vector<int> bit(sn.n_labels, -1);
  for (int i = 0; i < S; ++i) {
    sl[ordered[i]] = 1;
    bit[ordered[i]] = S - 1 - i;
  }
  const auto st = sym_run(sn, path, sl);
  const size_t n = sn.leaf.size();
  std::vector<uint64_t> dep(n + path.size(), 0);
  for (size_t i = 0; i < n; ++i)
    for (int x : sn.leaf[i])
      if (bit[x] >= 0) dep[i] |= 1ull << bit[x];
  for (size_t s = 0; s < path.size(); ++s) dep[n + s] = dep[path[s].first] | dep[path[s].second];
  // Runs of the step over all 2^S slices: in one sequence (the step reruns
  // whenever slice-id bit ctz(d) or a lower one changes), or dealt in
  // aligned windows of 2^w slices, each starting with everything computed
  // (2^(S-w) windows; a step independent of the window's bits runs once
  // per window).
  const int W = (window_bits > 0 && window_bits < S) ? window_bits : S;
  const int mb = std::min(merge_bits, W);
  if (mb > 0) {
    std::vector<std::pair<int, int>> kids(n + path.size(), {-1, -1});
    for (size_t s = 0; s < path.size(); ++s) kids[n + s] = {path[s].first, path[s].second};
    const MergeSets m = merge_sets(kids, dep, std::vector<char>(kids.size(), 0), mb);
    double f = 0;
    for (size_t s = 0; s + 1 < path.size(); ++s)
      f += (st[s].flops + launch_cost) * merge_runs(m.elig[n + s], m.emask[n + s], m.bmask[n + s], S, W);
    // the root adds every slice's value into the result: no accumulator of its own
    const size_t r = path.size() - 1;
    f += (st[r].flops + launch_cost) * merge_runs(m.elig[n + r], m.emask[n + r], 0, S, W);
    return f;
  }
  double f = 0;
  for (size_t s = 0; s < path.size(); ++s) {
    const uint64_t d = dep[n + s];
    const int lo = d ? __builtin_ctzll(d) : 64;
    double runs;
    if (W < S)
      runs = std::ldexp(lo >= W ? 1.0 : std::ldexp(1.0, W - lo), S - W);
    else
      runs = d ? std::ldexp(1.0, S - lo) : 1.0;
    f += (st[s].flops + launch_cost) * runs;
  }
  return f;
}

// Outer -> inner order: decreasing recomputation cost, i.e. the flops of all
// steps whose subtree holds a leaf carrying the index.  Inner (fast-varying)
// indices then force the least recomputation between consecutive slices.
std::vector<int> order_slices(const SymNet& sn, const Path& path, const std::vector<int>& sl) {
  std::vector<char> slm(sn.n_labels, 0);
  for (int x : sl) slm[x] = 1;
  auto st = sym_run(sn, path, slm);
  size_t n = sn.leaf.size();
  std::vector<std::pair<double, int>> cost;
  for (int x : sl) {
    std::vector<char> dep(n + path.size(), 0);
    for (size_t i = 0; i < n; ++i)
      dep[i] = std::binary_search(sn.leaf[i].begin(), sn.leaf[i].end(), x);
    double c = 0;
    for (size_t s = 0; s < path.size(); ++s) {
      dep[n + s] = dep[path[s].first] || dep[path[s].second];
      if (dep[n + s]) c += st[s].flops;
    }
    cost.push_back({-c, x});
  }
  std::stable_sort(cost.begin(), cost.end());
  std::vector<int> out;
  for (auto& p : cost) out.push_back(p.second);
  return out;
}

}  // namespace mitnc
