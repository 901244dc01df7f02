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
double reuse_total_flops(const SymNet& sn, const Path& path, const std::vector<int>& ordered, int window_bits = 0);
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
