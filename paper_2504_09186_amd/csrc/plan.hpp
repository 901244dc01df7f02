// Execution plan of a sliced contraction tree (host side).
#pragma once

#include <cstdint>
#include <vector>

#include "internal.hpp"
#include "step.hpp"

namespace mitnc {

constexpr int kLevelNever = 1000;   // node does not depend on any sliced index
constexpr int kLevelFirst = 1001;   // first slice of a range: everything runs
constexpr int kMergeClass = 7;      // timing slot of the post-lifetime merge additions
// Timing record of a merge addition: kMergeEvent - (4 * step + precision).
constexpr int kMergeEvent = -(1 << 30);
// Timing record of a batched forward SMALL launch of the range prologue: kFwdEvent - level.
constexpr int kFwdEvent = -(1 << 29);

struct PlanNode {
  bool leaf = false;
  int leaf_id = -1;
  std::vector<int64_t> labels;  // labels present after slicing
  std::vector<int> pos;         // physical address bit of each label
  std::vector<std::pair<int, int>> slice_bits;  // (slice-id bit, physical bit) of sliced labels
  int rank = 0;                 // labels.size()
  int full_rank = 0;            // address bits of the stored tensor (rank plus sliced bits kept, see hoisted)
  bool hoisted = false;         // computed once for all slices, sliced indices kept as ordinary ones
  uint64_t dmask = 0;           // slice-id bits this node depends on
  int lo = kLevelNever;         // recompute when a slice-id bit <= lo changes (lowest bit of emask)
  // Launch rule of SliceSchedule (internal.hpp): runs in slices with every
  // elig bit 1, when the emask bits change; bmask: merged slice-id bits
  // summed in this node's accumulator (post-lifetime merge).
  uint64_t elig = 0, emask = 0, bmask = 0;
  uint64_t tmp_offset = 0;      // accumulators: arena offset of the term being added
  int parent = -1;
  int region = 0;               // 0 leaf, 1 persistent, 2 transient, 3 result accumulator
  uint64_t offset = 0;          // byte offset inside the region (complex64 sizing)
  int exp = 0;                  // FP16/BF16 storage: value = mantissa * 2^exp
};

struct PlanStep {
  int a = -1, b = -1, out = -1;  // node ids; a is the larger operand
  bool swapped = false;
  bool root = false;
  int kclass = MITNC_K_SMALL;
  StepDesc d{};                  // pointer fields filled at launch
  StepDesc d64{};                // FP16/BF16 plans: complex64 geometry for calibration slices
  double flops = 0, bytes = 0;
  double flops_slice = 0, bytes_slice = 0;  // the same step within one slice (differs when hoisted)
  uint64_t part_bytes = 0;       // split-K partials, max over d and d64
};

// A fused stem section: consecutive steps of one chain run as one kernel.
// sd holds the tile maps and step descriptors; pointers, scales and the
// statistics slot are filled at launch.
struct PlanSection {
  std::vector<int> steps;        // plan step ids, chain order (the first step's A is the section input)
  SectionDesc sd{};
  double flops = 0, bytes = 0;   // summed step flops; algorithmic bytes of the fused pass
};

// One adjoint contraction of the reverse pass: for a step C = A (x) B the
// adjoint of A is the contraction of adj(C) with B onto A's indices.
struct RevOp {
  int step = -1;                 // forward step
  int target = -1;               // node whose adjoint is written
  int other = -1;                // forward value used (the target's sibling)
  bool adj_is_a = true;          // descriptor operand A is adj(C) (else the sibling)
  int kclass = MITNC_K_SMALL;
  StepDesc d{};
  uint64_t part_bytes = 0;
  double flops = 0;
};


}  // namespace mitnc

struct mitnc_plan {
  mitnc_plan_opts opts{};
  int n_leaves = 0;
  int S = 0;                                 // number of sliced indices
  std::vector<mitnc::PlanNode> nodes;        // leaves then step outputs
  std::vector<mitnc::PlanStep> steps;
  std::vector<mitnc::PlanSection> sections;  // fused stem sections
  std::vector<int> step_section;             // per step: section id or -1
  std::vector<std::vector<float>> leaf_data; // complex64 interleaved, full (unsliced) leaves
  std::vector<char> leaf_is_1q;              // leaf is a single-qubit gate
  std::vector<std::vector<uint32_t>> leaf_half;  // FP16/BF16 mantissas (precision plans)
  uint64_t leaf_bytes = 0, persist_bytes = 0, arena_bytes = 0, part_bytes = 0;
  // Workspace: [complex64 leaves | 16-bit leaves | persistent | arena |
  //             split-K partials | per-step maxima | calibration result]
  uint64_t off_leaf_half = 0, off_persist = 0, off_arena = 0, off_part = 0, off_stats = 0, off_calib = 0;
  uint64_t ws_bytes = 0;
  bool calibrated = false;
  int32_t reruns = 0;  // FP16/BF16 executes that re-ran after an exponent miss
  // The range prologue: the steps a slice range computes once (no sliced
  // operand index, or hoisted), run level by level before the range's first
  // slice (a level's steps read only leaves and outputs of earlier levels);
  // a level's SMALL steps go out in one launch through a table of workspace
  // offsets.  The arena keeps every prologue buffer distinct until the
  // prologue ends.  ftab64 holds the complex64 geometry for the calibration
  // slices of FP16/BF16 plans.
  struct FwdBatch {
    uint32_t first = 0, blocks = 0;  // block-table range of the level's batched SMALL steps
    double flops = 0, bytes = 0;
    std::vector<int> big;            // the level's other steps (launched one by one)
  };
  struct FwdRun {
    int first_step = -1, last_step = -1;
    std::vector<FwdBatch> levels, levels64;
  };
  std::vector<FwdRun> fwd_runs;
  std::vector<int> fwd_run_of;                // per step: its run or -1
  std::vector<mitnc::SmallFwdOp> ftab, ftab64;
  std::vector<int> ftab_step;                 // step of each ftab entry
  std::vector<uint32_t> fblock, fblock64;
  uint64_t off_ftab = 0, off_fblock = 0, off_ftab64 = 0, off_fblock64 = 0;
  int ftab_version = 0, ftab_uploaded = -1;   // out_scale changes since the table was copied
  std::vector<int> fwd_levels_tmp;            // plan construction: level of each run step's output
  std::vector<int> prologue_order;            // the prologue's steps, level by level
  // Post-lifetime merge: bits summed below the root; slice ranges must be
  // multiples of 2^merge_align_bits.
  uint64_t merged = 0;
  int merge_align_bits = 0;
  // Differentiation form (opts.differentiable): every node keeps its own
  // buffer, adjoints live in [off_adj, off_adj + adj_bytes).
  std::vector<char> has_grad;          // per node: a single-qubit gate leaf below
  std::vector<uint64_t> adj_offset;    // per node with has_grad
  std::vector<mitnc::RevOp> rev;       // reverse pass in execution order
  std::vector<mitnc::GradEntry> gtab;  // per single-qubit gate leaf
  // Reverse pass by depth: the ops of one level read adjoints written at
  // earlier levels only.  Each level runs its MFMA-class ops one by one and
  // all its SMALL ops in one launch over the block table entries
  // [small_first, small_first + small_blocks).
  struct RevLevel {
    std::vector<int> big;  // indices into rev
    uint32_t small_first = 0, small_blocks = 0;
  };
  std::vector<RevLevel> rev_levels;
  std::vector<int> rev_level_of;        // level of each rev entry
  // Grouped reverse pass: the reverse ops below a deferral root d (a kept
  // node whose sliced bits are all at or above lo(d)) are linear in adj(d)
  // and depend on the slice only through those bits, so adj(d) is summed
  // over each run of 2^lo(d) consecutive slices (the op writing it writes a
  // term buffer, added into the accumulator at adj_offset[d]) and the ops of
  // d's group run once per run.  Group 0 holds the ops above every deferral
  // root and runs for every slice.
  struct RevGroup {
    int root = -1;                 // deferral root node (-1: group 0)
    int lo = 0;                    // runs when the slice id is a multiple of 2^lo, or the range's first
    std::vector<RevLevel> levels;  // big ops and SMALL block-table ranges per reverse level
    std::vector<int> children;     // groups whose root's adjoint term this group writes
    uint32_t grad_first = 0, grad_count = 0;  // entries of gtab
  };
  std::vector<RevGroup> rev_groups;
  std::vector<uint64_t> adj_term_offset;  // per deferral root: its term buffer (offset in the adjoint region)
  std::vector<int> defer_group;           // per node: its group if it is a deferral root, else -1
  std::vector<int> rev_group_of;          // per rev entry: its group
  std::vector<mitnc::SmallRevOp> rtab;  // SMALL ops, uploaded at off_rtab
  std::vector<uint32_t> rblock;         // workgroup -> rtab entry, uploaded at off_rblock
  uint64_t off_rtab = 0, off_rblock = 0;
  int32_t n_grad_gates = 0;
  uint64_t off_adj = 0, adj_bytes = 0, off_gtab = 0;
  double rev_flops = 0;
  uint64_t result_elems = 0;
  int max_log2 = 0;
  bool uploaded = false;
  // Differentiable plans keep every node's value: the slice whose values the
  // workspace holds after the last forward pass (-1: none).
  int64_t valid_slice = -1;
  void* uploaded_ws = nullptr;
  // Optional per-launch timing (hipEvent pairs around each step's main kernel).
  bool timing = false;
  std::vector<void*> ev_pool;          // hipEvent_t
  size_t ev_used = 0;                  // pairs recorded since the last reset
  std::vector<int> ev_step;            // step index of each recorded pair
  ~mitnc_plan();
};

namespace mitnc {
mitnc_plan* build_plan(const mitnc_network* net, const mitnc_plan_opts& opts);
// Builds the descriptor and output layout of one step (operands P->nodes[st.a],
// P->nodes[st.b]; output labels c_labels, in root_layout order if given).
// Exponent e with max * 2^-e in [2^13, 2^14) (0 for max 0).
int mantissa_exponent(double max_abs);
void build_step_for(mitnc_plan* P, PlanStep& st, const std::vector<int64_t>& c_labels,
                    const std::vector<int64_t>* root_layout, int force_kernel, int precision);
}
