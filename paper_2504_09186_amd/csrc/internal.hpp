// Internal data structures of libmitnc (host side).
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/mitnc.h"

namespace mitnc {

using cd = std::complex<double>;

// Label of bit j of the batch hyperindex.
inline int64_t batch_label(int j) { return -1 - (int64_t)j; }
inline int64_t wire_label(int q, int t) { return (int64_t)q * 65536 + t; }

struct Leaf {
  std::vector<int64_t> labels;  // LSB first: address bit i carries labels[i]
  std::vector<cd> data;         // 2^labels.size() entries
  int32_t gate = -1;            // circuit gate index, -1 for state / projector leaves
  int32_t arity = 0;            // 1 or 2 for gate leaves
};

// Error with a status code; converted to a return value at the ABI.
struct Error {
  int32_t code;
  std::string msg;
};
[[noreturn]] void fail(int32_t code, const std::string& msg);

// Dense symbolic view of a network used by the planner: labels are renumbered
// 0..n_labels-1 and every tensor is a sorted vector of dense labels.
struct SymNet {
  int n_labels = 0;
  std::vector<int64_t> label_id;
  std::unordered_map<int64_t, int> dense;
  std::vector<std::vector<int>> leaf;
  std::vector<char> is_out;
  std::vector<char> closed;  // binary edge shared by exactly two leaves, not output
};

using Path = std::vector<std::pair<int32_t, int32_t>>;

// One step of a symbolic run over a path.
struct SymStep {
  int a, b;                 // operand node ids
  std::vector<int> c;       // output labels (sorted, dense)
  int c_bits = 0;           // log2 |C| (excluding sliced labels)
  int k_bits = 0;           // contracted bits
  double flops = 0;         // 8 * |C| * K
};

SymNet make_symnet(const std::vector<Leaf>& leaves, const std::vector<int64_t>& output);
// Runs the path symbolically with the given dense labels removed (sliced).
std::vector<SymStep> sym_run(const SymNet& sn, const Path& path, const std::vector<char>& sliced);
double sym_total_flops(const std::vector<SymStep>& st);
int sym_max_bits(const SymNet& sn, const std::vector<SymStep>& st, const std::vector<char>& sliced);
Path greedy_path(const SymNet& sn, double alpha, double temperature, uint64_t seed,
                 const std::vector<char>* removed = nullptr);
std::vector<int> greedy_slices(const SymNet& sn, const Path& path, int cap, int min_sliced,
                               int max_sliced, bool* ok);
std::vector<int> slice_reconf(const SymNet& sn, Path& path, const std::vector<int>& fixed, int cap, int min_sliced,
                              int max_sliced, int every, bool* ok);
double reuse_total_flops(const SymNet& sn, const Path& path, const std::vector<int>& ordered, int window_bits = 0,
                         int merge_bits = 0, double launch_cost = 0);
// Branch exchange (merge.cpp): local reordering of absorptions on chains,
// see the definition.  Returns the new path; *before / *after receive the
// reuse_total_flops of the old and new path.
Path branch_exchange(const SymNet& sn, const Path& path, const std::vector<int>& ordered, int window_bits,
                     int merge_bits, int cap_bits, int passes, double* before, double* after, double launch_cost = 0);

// Post-lifetime merge (merge.cpp).  Tree nodes 0..n-1 are leaves, then step
// outputs in path order (children before parents, the root last); kids[u] is
// {-1, -1} for a leaf.  dmask[u]: slice-id bits of the sliced indices carried
// by the leaves below u.  Bits below `candidate_bits` may be merged.
struct MergeSets {
  uint64_t merged = 0;            // merged bits summed below the root
  int align_bits = 0;             // slice ranges must be multiples of 2^align_bits
  std::vector<int> at;            // per slice-id bit: node whose parent takes the sum (-1: not merged)
  std::vector<uint64_t> elig;     // per node: bits that must all be 1 in a slice that computes it
  std::vector<uint64_t> emask;    // per node: bits its value (as its parent reads it) depends on
  std::vector<uint64_t> bmask;    // per node: bits summed in its accumulator (merged at this node)
};
MergeSets merge_sets(const std::vector<std::pair<int, int>>& kids, const std::vector<uint64_t>& dmask,
                     const std::vector<char>& hoisted, int candidate_bits);
// Computations of a node per 2^S slices run in aligned ranges of 2^W slices
// (W <= S) under the rule of SliceSchedule.
double merge_runs(uint64_t elig, uint64_t emask, uint64_t bmask, int S, int W);

// The per-slice launch rule shared by execution, the host replay check and
// the schedule query.  For slice s (slices of a range in increasing order):
// a node runs only if every bit of elig is 1 in s; it then runs if the bits
// emask & ~bmask differ from its last run (a new value: stored, or for an
// accumulator the first term of a new sum) or, for an accumulator, if the
// bits bmask of s form a pattern above the last term added to the current
// sum (the next term: added).  Slices in between that repeat an added
// pattern (a lower bit the node does not depend on changed) run nothing.
struct SliceSchedule {
  std::vector<uint64_t> key, pat;
  std::vector<char> seen;
  explicit SliceSchedule(size_t n_nodes) : key(n_nodes), pat(n_nodes), seen(n_nodes, 0) {}
  // 0: skip, 1: compute (store, or accumulate at the root), 2: compute and add into the accumulator.
  int decide(int node, uint64_t elig, uint64_t emask, uint64_t bmask, uint64_t s) {
    if ((s & elig) != elig) return 0;
    const uint64_t k = s & emask & ~bmask, p = s & bmask;
    if (!seen[node] || k != key[node]) {
      seen[node] = 1;
      key[node] = k;
      pat[node] = p;
      if (p != 0) fail(MITNC_INVALID_ARG, "internal: merge group starts at a nonzero pattern");
      return 1;
    }
    if (p > pat[node]) {
      pat[node] = p;
      return 2;
    }
    return 0;
  }
};
std::vector<int> order_slices(const SymNet& sn, const Path& path, const std::vector<int>& sl);
// Subtree reconfiguration (reconf.cpp): locally optimal re-ordering of the
// tree, flops measured with `removed` labels (sliced) absent, intermediates
// kept at most 2^cap_bits entries.
Path optimize_path(const SymNet& sn, const Path& path, const std::vector<char>* removed, int cap_bits, int passes);
void validate_path(int n_leaves, const Path& path);
// Recursive-bisection path search (partition.cpp).
struct PartitionParams {
  double imbalance = 0.1;   // part sizes within (1 +- imbalance) / 2 of the tensors split
  int cutoff = 8;           // parts of at most this many tensors are contracted greedily
  int starts = 4;           // initial cuts refined per bisection
  double ext_weight = 0.5;  // weight of cut indices also held outside the part
};
Path partition_path(const SymNet& sn, const std::vector<char>& removed, const PartitionParams& prm, uint64_t seed);

}  // namespace mitnc

struct mitnc_network {
  int32_t n_qubits = 0;
  std::vector<mitnc::Leaf> leaves;        // canonical leaf order
  std::vector<int32_t> segs;              // final segment index per qubit
  bool output_set = false;
  std::vector<int64_t> output_lsb;        // result layout, LSB first
  int32_t n_batch_bits = 0;
  mitnc::Path path;
  std::vector<int64_t> sliced;            // outer -> inner labels
};
