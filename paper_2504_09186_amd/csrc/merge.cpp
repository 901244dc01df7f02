// Post-lifetime merge and branch exchange (Sec. III-B).
//
// Pre-lifetime reuse keeps a node's value while the slice-id bits it depends
// on do not change.  After the lifetime of a sliced index ends (the node
// where both tensors carrying it have been contracted), everything above that
// node is linear in its value, so the two slices that differ only in that
// index can be merged: the node's values for index value 0 and 1 are summed
// in an accumulator and the rest of the tree runs once for the pair
// (distributivity of the contraction, Sec. III-B).  Combined with the
// pre-lifetime reuse this is the spindle of Sec. III-B.
//
// Here the merge is decided per slice-id bit b (bits below a candidate count,
// the innermost, fastest-varying ones):
//   * at[b]: the lowest non-hoisted node whose subtree holds every leaf
//     carrying b (where its lifetime ends);
//   * b is merged if every lower bit c that the subtree of at[b] depends on is
//     itself merged at at[b] or below it.  Slices run in increasing slice-id
//     order, so the terms of at[b]'s sum (b = 0, then 1, lower bits of the
//     subtree already summed) follow each other with nothing in between that
//     changes its other inputs: one accumulator per node suffices.  This is
//     the nesting condition of the spindle (an inner index's lifetime inside
//     an outer one's).
// Per node u: bmask(u) = bits merged at u (its accumulator sums over them);
// sum(u) = bits merged strictly below u (its inputs are already summed over
// them); emask(u) = bits its value depends on = dmask(u) minus sum(u);
// elig(u) = merged bits whose accumulator is not on the path from u to the
// root: a slice computes u only when all of them are 1, i.e. on the last
// slice of every such pair, where its parent can use the value.
//
// Branch exchange (Sec. III-B, last paragraph): when one tensor absorbs two
// others in consecutive steps, the two absorptions can be swapped without
// changing the result; doing so moves the start or end of lifetimes of the
// sliced indices the absorbed tensors carry, which changes the flops of the
// spindle.  The local search below swaps such pairs while that lowers the
// reuse-aware flops and keeps the size cap.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace mitnc {

MergeSets merge_sets(const std::vector<std::pair<int, int>>& kids, const std::vector<uint64_t>& dmask,
                     const std::vector<char>& hoisted, int candidate_bits) {
  const int n = (int)kids.size();
  MergeSets m;
  m.at.assign(64, -1);
  m.elig.assign(n, 0);
  m.bmask.assign(n, 0);
  m.emask.resize(n);
  for (int u = 0; u < n; ++u) m.emask[u] = hoisted[u] ? 0 : dmask[u];
  const int C = std::max(0, std::min(candidate_bits, 64));
  if (C == 0 || n == 0) return m;
  std::vector<int> parent(n, -1);
  for (int u = 0; u < n; ++u)
    if (kids[u].first >= 0) parent[kids[u].first] = parent[kids[u].second] = u;
  const int root = n - 1;
  // Leaves carrying each bit, and the lowest node holding all of them.
  std::vector<int> total(C, 0);
  std::vector<std::vector<int>> cnt(n, std::vector<int>(C, 0));
  for (int u = 0; u < n; ++u) {
    if (kids[u].first < 0) {
      for (int b = 0; b < C; ++b)
        if (dmask[u] >> b & 1) {
          cnt[u][b] = 1;
          total[b]++;
        }
    } else {
      for (int b = 0; b < C; ++b) cnt[u][b] = cnt[kids[u].first][b] + cnt[kids[u].second][b];
    }
  }
  std::vector<int> at(C, -1);
  for (int u = 0; u < n; ++u)
    for (int b = 0; b < C; ++b)
      if (at[b] < 0 && total[b] > 0 && cnt[u][b] == total[b]) at[b] = u;
  for (int b = 0; b < C; ++b)
    while (at[b] >= 0 && hoisted[at[b]]) at[b] = parent[at[b]];
  auto below_or_at = [&](int x, int y) {  // x in the subtree of y
    for (; x >= 0; x = parent[x])
      if (x == y) return true;
    return false;
  };
  uint64_t M = 0;
  for (int b = 0; b < C; ++b) {
    if (at[b] < 0) continue;
    bool ok = true;
    for (int c = 0; c < b && ok; ++c)
      if (dmask[at[b]] >> c & 1) ok = (M >> c & 1) && below_or_at(at[c], at[b]);
    if (ok) M |= 1ull << b;
  }
  for (int b = 0; b < C; ++b)
    if (M >> b & 1) {
      m.at[b] = at[b];
      m.bmask[at[b]] |= 1ull << b;
    }
  std::vector<uint64_t> sum(n, 0);
  for (int u = 0; u < n; ++u)
    if (kids[u].first >= 0) {
      const int a = kids[u].first, c = kids[u].second;
      sum[u] = sum[a] | m.bmask[a] | sum[c] | m.bmask[c];
    }
  m.elig[root] = sum[root];
  for (int u = root - 1; u >= 0; --u) m.elig[u] = parent[u] >= 0 ? m.elig[parent[u]] & ~m.bmask[u] : 0;
  for (int u = 0; u < n; ++u)
    if (!hoisted[u]) m.emask[u] = dmask[u] & ~sum[u];
  m.merged = M & ~m.bmask[root];
  m.align_bits = m.merged ? 64 - __builtin_clzll(m.merged) : 0;
  return m;
}

// Eligible slices of a node enumerate the bits outside elig in increasing
// order.  A new value (or, for an accumulator, a new sum) starts on the first
// one and whenever a bit of emask & ~bmask changes, i.e. 2^(number of
// non-elig bits at or above its lowest bit) times per range; an accumulator
// computes 2^|bmask| terms per sum.
double merge_runs(uint64_t elig, uint64_t emask, uint64_t bmask, int S, int W) {
  const uint64_t wm = W >= 64 ? ~0ull : (1ull << W) - 1;
  const uint64_t e = emask & ~bmask & wm;
  double per = std::ldexp(1.0, __builtin_popcountll(bmask & wm));
  if (e) {
    const int lo = __builtin_ctzll(e);
    const uint64_t free = wm & ~elig & ~((1ull << lo) - 1);
    per = std::ldexp(per, __builtin_popcountll(free));
  }
  return std::ldexp(per, S - W);
}

Path branch_exchange(const SymNet& sn, const Path& path0, const std::vector<int>& ordered, int window_bits,
                     int merge_bits, int cap_bits, int passes, double* before, double* after, double launch_cost) {
  Path path = path0;
  const int n = (int)sn.leaf.size();
  std::vector<char> sl(sn.n_labels, 0);
  for (int x : ordered) sl[x] = 1;
  double best = reuse_total_flops(sn, path, ordered, window_bits, merge_bits, launch_cost);
  if (before) *before = best;
  for (int pass = 0; pass < passes; ++pass) {
    bool improved = false;
    for (size_t s = 0; s + 1 < path.size(); ++s) {
      // step s: (x, b1) -> y = n + s; step s + 1 consumes y with b2.
      const int y = n + (int)s;
      const auto& p2 = path[s + 1];
      if (p2.first != y && p2.second != y) continue;
      const int b2 = p2.first == y ? p2.second : p2.first;
      // Either operand of step s may play b1: try both.
      for (int side = 0; side < 2; ++side) {
        Path trial = path;
        auto& t1 = trial[s];
        auto& t2 = trial[s + 1];
        int& b1 = side == 0 ? t1.second : t1.first;
        const int old_b1 = b1;
        b1 = b2;
        if (t2.first == y) t2.second = old_b1;
        else t2.first = old_b1;
        const auto st = sym_run(sn, trial, sl);
        if (sym_max_bits(sn, st, sl) > cap_bits) continue;
        const double f = reuse_total_flops(sn, trial, ordered, window_bits, merge_bits, launch_cost);
        if (f < best * (1 - 1e-12)) {
          best = f;
          path = std::move(trial);
          improved = true;
          break;
        }
      }
    }
    if (!improved) break;
  }
  if (after) *after = best;
  return path;
}

}  // namespace mitnc
