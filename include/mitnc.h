/*
 * mitnc: sliced tensor-network contraction of random quantum circuits on
 * AMD MI355X (gfx950).  C ABI of libmitnc.so.
 *
 * The calls follow the problem as the paper states it (SW-TNC, arXiv
 * 2504.09186): a circuit becomes a tensor network (Sec. II-A), a contraction
 * path orders the pairwise contractions (Sec. II-A; Evaluation), a set of
 * sliced indices splits the work into 2^s independent subtasks whose results
 * are summed (Sec. II-A, Sec. III-A), and the requested amplitudes are the
 * remaining open indices.
 *
 * General conventions
 *  - Every call returns an int32_t status: MITNC_OK (0) or a negative error
 *    code; mitnc_last_error() returns a thread-local message for the last
 *    failing call on the calling thread.  No C++ exception crosses the ABI.
 *  - Host objects (mitnc_network, mitnc_plan) are owned by the library and
 *    freed by the matching destroy call.
 *  - The library never allocates device memory.  The caller allocates the
 *    device workspace (size from mitnc_plan_query) and all device outputs;
 *    "device" pointers below must point to memory of the current HIP device.
 *  - "stream" is a hipStream_t passed as void* (NULL = default stream).  GPU
 *    calls are asynchronous on that stream.
 *  - Index (edge) labels are canonical: the wire segment of qubit q after its
 *    t-th gate (t = 0: after the initial |0>) has label q*65536 + t.
 *  - Leaf (tensor) ids are canonical: gate instances in circuit order, then
 *    the initial-state leaf of each qubit 0..n-1, then one output projector
 *    leaf for each fixed or batched qubit in increasing qubit order.
 *  - Result order: batch index (if any) most significant, then the open
 *    qubits in increasing qubit order (lower qubit = more significant bit).
 */
#ifndef MITNC_H
#define MITNC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MITNC_OK = 0,
  MITNC_INVALID_ARG = -1,
  MITNC_PATH_INVALID = -2,
  MITNC_WORKSPACE_TOO_SMALL = -3,
  MITNC_HIP_ERROR = -4,
  MITNC_UNSUPPORTED = -5,
  MITNC_NUMERIC = -6
};

enum { MITNC_C64 = 0, MITNC_CF16 = 1, MITNC_CBF16 = 2 };

typedef struct mitnc_network mitnc_network;
typedef struct mitnc_plan mitnc_plan;

/* One gate instance.  arity 1 or 2; q1 ignored for arity 1.  mat points to
 * the complex128 matrix U[out][in], interleaved (re, im), row-major, 2x2 or
 * 4x4; for two qubits the row/column index is (bit of q0)*2 + (bit of q1).
 * The matrix is copied. */
typedef struct mitnc_gate {
  int32_t arity;
  int32_t q0, q1;
  const double* mat;
} mitnc_gate;

/* Circuit -> tensor network (Sec. II-A: gates are the nodes, wire segments
 * the edges; initial state |0...0>).  Every gate instance becomes its own
 * leaf.  Errors: INVALID_ARG for bad qubits, arity or null pointers. */
int32_t mitnc_network_from_circuit(int32_t n_qubits, int32_t n_gates, const mitnc_gate* gates,
                                   mitnc_network** out);

/* Requested amplitudes.  per_qubit[q]: 0 or 1 = fixed output bit, -1 = open,
 * -2 = batched.  batch_bits: n_batch x (number of batched qubits) bytes
 * (0/1), row-major, batched qubits in increasing order; n_batch must be a
 * power of two (the batch index is a set of log2(n_batch) binary hyper-
 * indices) and may be 0 if no qubit is batched.  Must be called exactly once
 * before any path call. */
int32_t mitnc_network_set_output(mitnc_network* net, const int8_t* per_qubit, int32_t n_batch,
                                 const uint8_t* batch_bits);

/* Sizes of the network of Sec. II-A: n_leaves receives the number of
 * tensors (a contraction path has n_leaves - 1 steps), n_labels (may be
 * NULL) the number of distinct indices.  Errors: INVALID_ARG for a null
 * network. */
int32_t mitnc_network_info(const mitnc_network* net, int32_t* n_leaves, int32_t* n_labels);

/* Contraction order and slicing search.  Runs `trials` randomised greedy
 * paths (the first one unperturbed; pair cost size(out) - alpha *
 * (size(a) + size(b)), perturbed by Gumbel noise), slices each greedily
 * until the largest intermediate is <= 2^max_log2_elems and at least
 * min_sliced indices are sliced (at most max_sliced), and keeps the path and
 * slicing with the lowest total flops.  Sliced indices are ordered
 * outer -> inner by decreasing recomputation cost, which is the slice-id
 * bit order (the last one is the least significant bit).  The paper's index
 * overhead O(a) = 2 C_a / C_ori (Eq. 1) is reported by
 * mitnc_index_overhead.  Errors: UNSUPPORTED if the cap cannot be met within
 * max_sliced. */
typedef struct mitnc_search_opts {
  uint64_t seed;
  int32_t trials;
  int32_t max_log2_elems;
  int32_t min_sliced;
  int32_t max_sliced;
  int32_t keep_slicing; /* 1: keep the current sliced indices (outermost, in
                           their order) and only add more if the cap needs it */
  int32_t method;       /* 0: randomised greedy trials; 1: recursive-bisection
                           trials (parts sharing few indices, refined by
                           Fiduccia-Mattheyses moves, random balance and
                           leaf-size parameters per trial); 2: both, `trials`
                           of each */
  int32_t window_bits;  /* methods 1 and 2 rank trials by the flops all
                           slices execute with shared-prefix reuse (Sec.
                           III-B): run in one sequence (0), or dealt in
                           aligned ranges of 2^window_bits slices (one per
                           device or stream), each range starting cold */
  int32_t merge_bits;   /* methods 1 and 2: the ranking also counts the
                           post-lifetime merge of the innermost merge_bits
                           slice-id bits (mitnc_plan_opts.merge_bits; 0..12) */
  int32_t branch_exchange; /* 1: after the search, reorder absorptions
                              (mitnc_branch_exchange) with the same ranking */
  double launch_cost_flops; /* methods 1 and 2 (and branch exchange): added to
                               the ranking for every step computation, in
                               flops (0: flops only); a stand-in for the
                               fixed cost of a kernel launch, which decides
                               workloads of many small steps */
} mitnc_search_opts;
int32_t mitnc_path_search(mitnc_network* net, const mitnc_search_opts* opts);

/* Contraction path (Sec. II-A: the order of the pairwise contractions;
 * Evaluation: the paper takes it from an external search) as SSA pairs:
 * step t contracts ids pairs[2t], pairs[2t+1] into id n_leaves + t.
 * Errors: INVALID_ARG for null pointers, PATH_INVALID for a path that
 * reuses or skips a tensor.  get: pairs_out has room for 2*(n_leaves-1) int32.
 * set: validates (every id used once, ids exist when used).  Setting a path
 * keeps the slicing. */
int32_t mitnc_get_path(const mitnc_network* net, int32_t* pairs_out);
int32_t mitnc_set_path(mitnc_network* net, int32_t n_steps, const int32_t* pairs);

/* Sliced indices (Sec. III-A: fixing an index splits the contraction into
 * independent subtasks whose results are summed), outer -> inner (the last
 * is the least significant bit of the slice id; slices run in increasing id
 * order, so inner indices change most often, Sec. III-B).  get: n_out receives the count; ids_out (may be NULL) has
 * room for 64 labels.  set: every label must be a closed binary edge (shared
 * by exactly two leaves, not an output). */
int32_t mitnc_get_slicing(const mitnc_network* net, int32_t* n_out, int64_t* ids_out);
int32_t mitnc_set_slicing(mitnc_network* net, int32_t n, const int64_t* ids);

/* Greedy slicing for the current path (Sec. III-A; the same rule as
 * mitnc_path_search): slices indices until the largest intermediate has at
 * most 2^max_log2_elems entries and at least min_sliced indices are sliced
 * (at most max_sliced <= 64), replacing the current slicing.  n_out and
 * ids_out (room for 64 labels) receive the chosen labels, outer -> inner;
 * either may be NULL.  Errors: UNSUPPORTED if the cap cannot be met within
 * max_sliced (the slicing is then unchanged). */
int32_t mitnc_slice_greedy(mitnc_network* net, int32_t max_log2_elems, int32_t min_sliced,
                           int32_t max_sliced, int32_t* n_out, int64_t* ids_out);

/* Eq. (1) of the paper for label `a` on the current path and slicing:
 * O(a) = 2 C_a / C_ori, C = real flops of one subtask (8 per complex
 * multiply-add).  Host only. */
int32_t mitnc_index_overhead(const mitnc_network* net, int64_t label, double* overhead);

/* Branch exchange (Sec. III-B, last paragraph): where one tensor absorbs two
 * others in consecutive steps, swapping the two absorptions leaves the
 * result unchanged but moves where lifetimes of sliced indices start and
 * end.  Local search over such adjacent pairs of the current path (up to
 * `passes` sweeps), keeping each swap that lowers the flops of all slices
 * with pre-lifetime reuse and the post-lifetime merge of the innermost
 * merge_bits bits (ranges of 2^window_bits slices as in mitnc_search_opts),
 * plus launch_cost_flops per step computation (as in mitnc_search_opts),
 * and keeps every intermediate within 2^max_log2_elems entries; replaces
 * the path, keeps the slicing.  flops_before / flops_after (either may be
 * NULL) receive that count for the old and new path.  Host only.  Errors:
 * INVALID_ARG (no path, bad argument). */
int32_t mitnc_branch_exchange(mitnc_network* net, int32_t window_bits, int32_t merge_bits, int32_t max_log2_elems,
                              int32_t passes, double launch_cost_flops, double* flops_before, double* flops_after);

/* Plan options.  precision: MITNC_C64 (complex64 storage, FP32 arithmetic on
 * MFMA) or MITNC_CF16 / MITNC_CBF16 (each tensor stored as complex FP16 or
 * BF16 mantissas with a power-of-two exponent per tensor, contractions on
 * FP16/BF16 MFMA with FP32 accumulation, FP64 cross-slice sum; requires
 * mitnc_calibrate after upload); reuse: 1 = recompute a tree node only when
 * the sliced indices below it change between consecutive slices (Sec. III-B,
 * pre-lifetime reuse), and contract small subtrees that depend on sliced
 * indices once for all slices, keeping those indices (at most 2^14 entries
 * per intermediate; not in differentiable plans), 0 = recompute every node
 * for every slice;
 * cache_budget_bytes: maximum device bytes of tensors kept across slices
 * (0 = unlimited; Sec. III-B dynamic tuning demotes the largest cached
 * tensors); force_kernel: -1 = automatic kernel choice, otherwise a kernel
 * class id (testing aid). */
typedef struct mitnc_plan_opts {
  int32_t precision;
  int32_t reuse;
  uint64_t cache_budget_bytes;
  int32_t force_kernel;
  int32_t differentiable; /* 1: keep every node's value for the reverse pass
                             (mitnc_backward); complex64 only */
  int32_t fuse_sections;  /* 1: run chains of steps that contract one large tensor
                             with small ones as fused sections (Sec. IV: the
                             tensor's tile stays in LDS across the chain);
                             ignored with force_kernel >= 0 or differentiable.
                             0 (recommended on MI355X): one stream launch per
                             step, which measured faster */
  int32_t no_rerun;       /* FP16/BF16 plans: 1 = an exponent miss or overflow
                             makes mitnc_execute return MITNC_NUMERIC at once;
                             0 = it re-derives the exponents and re-runs */
  int32_t splitk_max_mn_bits; /* split-K GEPDOT (Sec. V-B) takes steps whose m
                                 and n index counts are both at most this
                                 (0 = 4, i.e. M, N <= 16; at most 8) */
  int32_t splitk_target_bits; /* log2 of the workgroups (waves for the
                                 register-only form) a split-K step is spread
                                 over, K split until the grid reaches it
                                 (0 = 12 register-only, 11 LDS-tiled, 9 for
                                 the large TILE and TALL tiles; at most 16) */
  int32_t merge_bits;         /* post-lifetime merge (Sec. III-B, with the
                                 pre-lifetime reuse: the spindle): 0 = off;
                                 k = the k innermost slice-id bits (0..12) may
                                 be merged.  Bit b is merged when the node
                                 where its index's lifetime ends (lowest
                                 non-hoisted node holding both tensors that
                                 carry it) depends on no lower bit that is not
                                 merged at or below that node (nested
                                 lifetimes).  That node then sums its values
                                 for b = 0 and 1 in a kept accumulator, and
                                 the steps above it run once per pair.  Slice
                                 ranges of mitnc_execute must then be
                                 multiples of 2^merge_align_bits (stats).
                                 Requires reuse; not with differentiable or
                                 fuse_sections (UNSUPPORTED) */
  int32_t no_hoist;           /* 1: small subtrees that depend on sliced
                                 indices are not hoisted (contracted once for
                                 all slices); they then run per slice under
                                 the reuse rule like every other node */
  int32_t prologue_bits;      /* forward steps computed once per slice range
                                 run first, level by level, SMALL ones
                                 batched into one launch per level (the range
                                 prologue).  0: steps with no sliced index
                                 (or hoisted); w > 0: also steps whose sliced
                                 indices are all at slice-id bits >= w, and
                                 ranges must then lie in one aligned block of
                                 2^w slices (at most 62) */
  int32_t reverse_defer;      /* differentiable plans, grouped reverse pass:
                                 the reverse below a kept node d depends on
                                 the slice only through d's sliced bits (all
                                 at or above its lowest, lo), so adj(d) is
                                 summed over each run of 2^lo slices and the
                                 adjoint ops below d run once per run.
                                 0: at the kept nodes where a cost model
                                 (flops saved against the added accumulation
                                 traffic) expects a gain; 1: at every kept
                                 node; -1: never */
} mitnc_plan_opts;

/* Execution plan of the sliced contraction tree for the network's current
 * path and slicing (Sec. II-A, III-A, III-B): per step the kernel class,
 * operand address maps (the permutation of TTGT as an address map, Sec.
 * V-A), output layout, split-K factor (Sec. V-B), per-node recompute level
 * and the workspace layout.  Host only; the plan copies what it needs from
 * the network.  Errors: INVALID_ARG (null, bad option), UNSUPPORTED (a
 * step outside every kernel class, or more than 64 sliced indices). */
int32_t mitnc_plan_create(const mitnc_network* net, const mitnc_plan_opts* opts, mitnc_plan** out);

/* Sizes and algorithmic work of a plan (host only).  Flops count 8 real
 * flops per complex multiply-add (the 4M convention, whatever split runs);
 * bytes count every operand read once and every output written once.
 * Errors: INVALID_ARG for null pointers. */

typedef struct mitnc_plan_stats {
  uint64_t workspace_bytes;   /* device bytes the caller must provide */
  uint64_t result_elems;      /* complex entries of the result */
  int32_t n_sliced;           /* S: slice ids are 0 .. 2^S - 1 */
  int32_t n_steps;            /* contraction steps per full slice */
  int32_t max_log2_elems;     /* largest intermediate */
  int32_t n_kernel_classes;
  double flops_full_slice;    /* real flops of one slice without reuse or hoisting */
  double flops_reused_slice;  /* average real flops per slice actually executed over 2^S slices
                                 (reuse of unchanged subtrees, hoisted subtrees run once) */
  double bytes_full_slice;    /* algorithmic HBM bytes of one slice without reuse */
  double bytes_reused_slice;
  int32_t steps_by_class[8];  /* step count per kernel class */
  double flops_by_class[8];   /* full-slice flops per kernel class */
  int32_t n_grad_gates;       /* differentiable plans: single-qubit gates (gradient entries / 4) */
  int32_t n_reverse_ops;      /* adjoint contractions per slice */
  double flops_reverse_slice; /* real flops of the reverse pass of one slice */
  int32_t n_merged;           /* slice-id bits merged below the root (merge_bits) */
  int32_t merge_align_bits;   /* execute ranges must be multiples of 2^this (0: any) */
  uint64_t merged_mask;       /* the merged bits */
  int32_t n_reverse_groups;   /* differentiable plans: deferral roots of the grouped reverse pass */
  int32_t n_batched_small;    /* forward steps of the range prologue (computed once per slice
                                 range, run first level by level; see prologue_bits) */
  int32_t n_batched_launches; /* the batched launches of its SMALL steps (one per level) */
} mitnc_plan_stats;
int32_t mitnc_plan_query(const mitnc_plan* plan, mitnc_plan_stats* stats);

/* Per-step description for reports (host only; the per-step costs behind
 * Eq. (1) and the kernel classes of Sec. V).  info has 12 doubles per
 * step: kernel class, m bits, n bits, k bits, batch bits, recompute level
 * (-1 = slice invariant), flops, algorithmic bytes, k-split count, swapped,
 * output log2 size, is-root. */
int32_t mitnc_plan_steps(const mitnc_plan* plan, double* info);

/* Introspection of a plan's address maps and schedule (host only; used to
 * re-execute a plan independently on the host and to inspect layouts).
 * Nodes: leaves 0 .. n_leaves-1 in canonical order, then the output of step
 * s is node n_leaves + s.  A node's tensor is a flat array whose address
 * bits are binary indices (Sec. V-A); a step computes
 *   C[b, m, n] = sum_k A[b, m, k] B[b, k, n]
 * with logical bit i of m at address bit am[i] of A and cm[i] of C, and so
 * on (TTGT with the permutation applied as an address map, Sec. II-A).
 * Errors: INVALID_ARG for a null pointer or an id out of range. */
typedef struct mitnc_step_info {
  int32_t a, b, out;               /* node ids; a is the larger operand */
  int32_t root;                    /* 1: adds C into the complex128 result */
  int32_t kernel_class;
  int32_t section;                 /* fused section id, or -1 */
  int32_t section_pos, section_len;/* place in the section; the whole section
                                      runs when its last step is reached, and
                                      only its last output is stored */
  int32_t mb, nb, kb, bb;          /* bit counts of m, n, k and batch */
  uint8_t am[32], ak[32], ab[32];  /* A address bit of each m, k, batch bit */
  uint8_t bk[32], bn[32], bbt[32]; /* B address bit of each k, n, batch bit */
  uint8_t cm[32], cn[32], cb[32];  /* C address bit of each m, n, batch bit */
  /* MFMA-class steps (kernel class TILE, TALL, SPLITK; zero otherwise): */
  int32_t tm, tn, tk;              /* tile bits of m, n, k */
  uint8_t a_tile[16], b_tile[16];  /* tile bits of A / B in address order:
                                      class << 5 | index, class 0 m, 1 k, 2 n */
  uint8_t lds_a_swz[8], lds_b_swz[8]; /* complex64: LDS row k of the A (B) stage
                                      stores column c at c ^ XOR of swz[j]
                                      over the set bits j of k */
  uint16_t lds_a_row[8], lds_b_row[8]; /* FP16/BF16: LDS word address vector
                                      of A row bit i (m bit i) and of the
                                      expanded B row bit r (r = 0 re/im row,
                                      r = i + 1 n bit i) */
  uint8_t lds_k_col[8];            /* FP16/BF16: LDS column bit of tile k bit j;
                                      a tile entry's word address is the XOR
                                      of its bits' vectors */
  int32_t vec_a, vec_b;            /* FP16/BF16: 16-byte loads planned (4) or not (1) */
} mitnc_step_info;
int32_t mitnc_plan_step_info(const mitnc_plan* plan, int32_t step, mitnc_step_info* info);

/* Reverse pass of a differentiable plan (the adjoint contractions of
 * mitnc_backward): n_ops receives the number of adjoint contractions; with
 * info non-NULL, op (0 <= op < n_ops, execution order) is described in the
 * step_info layout: a = node whose adjoint is read, b = forward value it is
 * contracted with, out = node whose adjoint is written, root = the reverse
 * level (ops of one level are independent; SMALL ops of a level share one
 * launch), section = -1.  Errors: INVALID_ARG for a null plan or op out of
 * range; n_ops = 0 for plans that are not differentiable.  Host only. */
int32_t mitnc_plan_reverse_info(const mitnc_plan* plan, int32_t op, mitnc_step_info* info, int32_t* n_ops);

/* Storage and schedule of one node (host only; Sec. III-B reuse levels).
 * ws_offset: byte offset of the node's tensor in the workspace of a
 * complex64 run (UINT64_MAX for the root, which is the caller's result);
 * level: the lowest bit of recompute_mask, -1 if it is empty; without
 * merged bits a node is recomputed for slice s when ctz(s) >= level and
 * once per slice range for -1 (Sec. III-B; the masks below give the
 * general rule); a slice reads the sub-tensor at
 * element offset sum_j ((s >> slice_bit[j]) & 1) << slice_pos[j] (sliced
 * leaves and hoisted results; the step that writes a hoisted result writes
 * all 2^full_rank entries). */
typedef struct mitnc_node_info {
  int32_t is_leaf;
  int32_t rank;                    /* address bits seen by one slice */
  int32_t full_rank;               /* address bits stored */
  int32_t level;
  int32_t hoisted;                 /* contracted once for all slices */
  int32_t n_slice_bits;
  int32_t slice_bit[64];
  int32_t slice_pos[64];
  uint64_t ws_offset;
  /* Launch rule (Sec. III-B pre- and post-lifetime reuse), slices of a range
   * in increasing order: the node runs only in slices whose elig_mask bits
   * are all 1; then when the bits recompute_mask & ~merge_mask differ from
   * its last run (a new value: stored) or, for a merge accumulator
   * (merge_mask != 0), when the merge_mask bits differ (the next term:
   * computed into the buffer at merge_tmp_offset, then added). */
  uint64_t elig_mask;
  uint64_t recompute_mask;
  uint64_t merge_mask;
  uint64_t merge_tmp_offset;       /* workspace byte offset (accumulators) */
} mitnc_node_info;
int32_t mitnc_plan_node_info(const mitnc_plan* plan, int32_t node, mitnc_node_info* info);

/* The launches mitnc_execute makes for slices [slice_begin, slice_end), in
 * order, as (slice, step, mode) triples of int64: mode 1 = the step runs
 * and stores its output (the root step adds into the result), mode 2 = the
 * step runs into its node's merge buffer and the buffer is added into the
 * node's accumulator (post-lifetime merge, Sec. III-B).  Steps of a fused
 * section are listed at their own positions.  Writes at most `capacity`
 * triples to ops_out (may be NULL with capacity 0); *n_ops receives the
 * total count.  Host only.  Errors: INVALID_ARG (null n_ops, bad range,
 * range not aligned to 2^merge_align_bits). */
int32_t mitnc_plan_schedule(const mitnc_plan* plan, uint64_t slice_begin, uint64_t slice_end, int64_t capacity,
                            int64_t* ops_out, int64_t* n_ops);

/* The complex64 entries (re, im interleaved) a plan uploads for leaf
 * `leaf` (a gate tensor of Sec. II-A in its address layout; sliced leaves
 * hold every value of their sliced indices): 2^full_rank entries; out may
 * be null to query n_floats.  Host only.  Errors: INVALID_ARG (null, leaf
 * out of range, capacity too small). */
int32_t mitnc_plan_leaf_data(const mitnc_plan* plan, int32_t leaf, float* out, uint64_t capacity_floats,
                             uint64_t* n_floats);

/* Copies leaves and tables into the caller-owned device workspace (ws,
 * ws_bytes >= workspace_bytes; the workspace stays the caller's and must
 * outlive every later call on this plan) and resets the cross-slice cache
 * (Sec. III-B) and, for FP16/BF16 plans, the calibration.  Synchronises
 * the stream.  Errors: INVALID_ARG (null), WORKSPACE_TOO_SMALL, HIP_ERROR. */
int32_t mitnc_plan_upload(mitnc_plan* plan, void* ws, size_t ws_bytes, void* stream);

/* Contracts slices slice_begin .. slice_end-1 in order and ADDS their sum to
 * result_accum (device, complex128 interleaved, result_elems entries; FP64
 * cross-slice sum, Sec. VI: the single reduction of the method; slices are
 * independent subtasks, Sec. III-A, and a node is recomputed only when a
 * sliced index below it changes, Sec. III-B).  Must follow
 * mitnc_plan_upload on the same workspace (and, for FP16/BF16 plans,
 * mitnc_calibrate).  Complex64 plans: asynchronous on `stream`.
 * FP16/BF16 plans (value = mantissa * 2^e per tensor): the slices are
 * summed in a workspace buffer first; the call then synchronises the stream
 * and checks every stored step's largest |Re|, |Im|: a non-finite value, a
 * value >= 65504 with FP16 storage, or a largest value outside
 * [2^9, 2^18) (more than 2^4 away from the target [2^13, 2^14)) is an
 * overflow or exponent miss.  On a miss the exponents are re-derived from
 * complex64 maxima over this slice range (as mitnc_calibrate) and the range
 * runs once more; only a clean run is added to result_accum.  Errors:
 * INVALID_ARG for an empty or out-of-range slice range (with merged bits:
 * also one whose ends are not multiples of 2^merge_align_bits; with
 * prologue_bits > 0, one that leaves an aligned block of 2^prologue_bits
 * slices) or an
 * uncalibrated FP16/BF16 plan, WORKSPACE_TOO_SMALL, HIP_ERROR, NUMERIC when
 * the re-run misses again or the plan was created with no_rerun
 * (result_accum is then unchanged). */
int32_t mitnc_execute(mitnc_plan* plan, void* ws, size_t ws_bytes, uint64_t slice_begin,
                      uint64_t slice_end, double* result_accum, void* stream);

/* FP16/BF16 plans (not in the paper; the precision form): chooses every
 * stored tensor's power-of-two exponent.  Runs slices slice_begin ..
 * slice_end-1 in complex64 inside the workspace, records each step's
 * largest |Re|, |Im| and sets the exponent so that this maximum maps into
 * [2^13, 2^14) (two bits of headroom below the FP16 maximum); a step that
 * was all zero gets the worst-case exponent e_A + e_B + 14 + (contracted
 * bits).  Slices are statistically alike, so one or a few slices suffice;
 * mitnc_execute corrects a miss.  With merged bits the range is widened to
 * whole merge groups; it must then lie in one aligned block of
 * 2^prologue_bits slices if prologue_bits > 0.  Synchronises the stream.
 * No effect on complex64 plans.  Errors: INVALID_ARG (range),
 * WORKSPACE_TOO_SMALL, HIP_ERROR. */
int32_t mitnc_calibrate(mitnc_plan* plan, void* ws, size_t ws_bytes, uint64_t slice_begin,
                        uint64_t slice_end, void* stream);

/* FP16/BF16 plans: per step, the largest stored |Re|, |Im| (after scaling,
 * before rounding to 16 bits; +inf for a non-finite value) of the last
 * mitnc_execute call (of its final run).  Copies n_steps floats to host
 * memory `out` (synchronises the stream) and clears them if reset != 0.
 * Errors: INVALID_ARG, WORKSPACE_TOO_SMALL, HIP_ERROR. */
int32_t mitnc_step_maxima(mitnc_plan* plan, void* ws, size_t ws_bytes, float* out, int32_t reset,
                          void* stream);

/* FP16/BF16 plans: per-node exponents (node ids as in mitnc_plan_node_info:
 * leaves, then step outputs; value = stored mantissa * 2^exp) and the
 * number of exponent re-runs mitnc_execute has made.  exps_out (n_leaves +
 * n_steps int32, may be NULL) receives the current exponents; exps_in (may
 * be NULL) replaces those of the step outputs (leaf entries are ignored,
 * their mantissas were fixed at plan creation) and the scale factors of the
 * steps follow.  A testing and inspection aid: a wrong exponent is caught
 * and corrected by mitnc_execute.  Host only.  Errors: INVALID_ARG. */
int32_t mitnc_plan_exponents(mitnc_plan* plan, int32_t* exps_out, const int32_t* exps_in, int32_t* reruns_out);

/* Differentiation form (not in the paper; the problem is: loss
 * L = sum_b log|a_b|^2 over a batch of amplitudes, gradients with respect to
 * every single-qubit gate instance, each an independent complex 2x2
 * parameter).  This call computes the holomorphic vector-Jacobian product
 *   grad[g][i][j] += sum_r w[r] * d result[r] / d U_g[i][j]
 * summed over slices slice_begin .. slice_end-1, where result[r] is the
 * (partial) amplitude sum mitnc_execute would give for those slices and
 * U_g[i][j] (U[out][in]) enters linearly; no conjugation is applied (for L,
 * w = 1 / a, and dL/dRe U + i dL/dIm U = 2 conj(grad)).  Method, per slice:
 * recompute the forward contraction (nodes whose sliced indices did not
 * change are reused, Sec. III-B), seed the root's adjoint with w, and for
 * every step C = A (x) B with a single-qubit gate leaf below, adj(A) +=
 * adj(C) contracted with B onto A's indices (the same kind of pairwise
 * contraction, batch indices kept; likewise for B); subtrees without such
 * leaves are pruned.  The adjoint contractions run level by level of the
 * reverse tree (mitnc_plan_reverse_info); the SMALL ones of a level share
 * one launch.  A sliced gate leaf's adjoint goes to the entries of its
 * sliced values.  grad_accum: device complex128, n_grad_gates x 4 entries,
 * gates in circuit order of the single-qubit gates.  w: device complex128,
 * result_elems entries in result order.  Needs a plan created with
 * differentiable = 1 and uploaded.  Asynchronous on `stream`.  Errors:
 * INVALID_ARG (not differentiable, range, null), WORKSPACE_TOO_SMALL,
 * HIP_ERROR. */
int32_t mitnc_backward(mitnc_plan* plan, void* ws, size_t ws_bytes, uint64_t slice_begin,
                       uint64_t slice_end, const double* w, double* grad_accum, void* stream);

/* Differentiation form: replaces the matrices of all single-qubit gates of
 * an uploaded plan (the parameters of mitnc_backward; host complex128,
 * n_grad_gates x 4 entries U[out][in], circuit order) and re-uploads those
 * leaves (a sliced leaf keeps every value of its sliced indices); the
 * cross-slice cache restarts at the next execute.  Complex64 plans only.
 * Synchronises the stream.  Errors: INVALID_ARG (null, not uploaded,
 * precision), HIP_ERROR. */
int32_t mitnc_plan_set_gates(mitnc_plan* plan, void* ws, size_t ws_bytes, const double* mats,
                             void* stream);

/* Single pairwise contraction on the GPU (the TTGT step of Sec. II-A /
 * Sec. V with the permutation fused into the loads; split-K for long
 * common indices, Sec. V-B).  A, B, C: device
 * tensors of 2^ra, 2^rb, 2^rc complex entries (precision MITNC_C64:
 * interleaved float; MITNC_CF16 / MITNC_CBF16: interleaved 16-bit halves)
 * whose address bit i carries label la[i] / lb[i] / lc[i].  Labels shared by
 * A and B and absent from C are summed; labels in all three are batch
 * labels; every other label must appear in exactly one operand and in C.  C
 * is overwritten with the result times out_scale (use 1 for complex64).
 * work/work_bytes: device scratch for split-K partials (may be NULL/0 when no
 * split is needed; call with A, B and C all NULL to get the size in
 * *work_bytes_needed).  kernel: -1 automatic, else a class id.  Errors:
 * INVALID_ARG for inconsistent labels. */
int32_t mitnc_contract(const void* A, int32_t ra, const int64_t* la, const void* B, int32_t rb,
                       const int64_t* lb, void* C, int32_t rc, const int64_t* lc, int32_t precision,
                       float out_scale, int32_t kernel, void* work, size_t work_bytes,
                       size_t* work_bytes_needed, void* stream);

/* Allocation-free form of mitnc_contract, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the split-K partial sums live in a
 * fixed device array of MITNC_NOALLOC_SCRATCH_BYTES inside the library, one
 * per GPU, held until the process ends (its device address is looked up on
 * the first call on each device).  The caller passes inputs and output only;
 * the call allocates and frees nothing.  A step whose partials would need
 * more than the array fails with WORKSPACE_TOO_SMALL (use mitnc_contract
 * with a work buffer).  Every call on one GPU shares the array and leaves its
 * partials there: calls that overlap on one GPU (other streams or threads)
 * race and must be serialised by the caller.  Nothing needs clearing: every
 * partial a call reads, it has written first.  Same arguments, results and
 * other errors as mitnc_contract. */
#define MITNC_NOALLOC_SCRATCH_BYTES (32u << 20)
int32_t mitnc_contract_noalloc(const void* A, int32_t ra, const int64_t* la, const void* B, int32_t rb,
                               const int64_t* lb, void* C, int32_t rc, const int64_t* lc, int32_t precision,
                               float out_scale, int32_t kernel, void* stream);

/* Launch timing for measurement (the per-kernel figures of the paper's
 * performance analysis, Sec. VII).  mitnc_plan_timing(plan, 1) starts
 * recording a hipEvent pair around the main kernel of every step launched by
 * mitnc_execute (events are created on first use and reused after a reset);
 * calling it again (enable 0 or 1) discards the recorded pairs.
 * mitnc_plan_timing_read waits for the recorded events and fills, per kernel
 * class (8 entries each; entry 6 = fused sections, entry 7 = the additions
 * of the post-lifetime merge): summed kernel milliseconds, launch count, and
 * the algorithmic real flops and HBM bytes of those launches (for a section:
 * its input, small tensors and output; for a merge addition: the
 * accumulator read and written and the term read). */
int32_t mitnc_plan_timing(mitnc_plan* plan, int32_t enable);
int32_t mitnc_plan_timing_read(mitnc_plan* plan, double* ms, double* launches, double* flops,
                               double* bytes);

/* Frees a plan or network (host memory only; NULL is ignored).  A plan does
 * not reference its network after mitnc_plan_create. */
void mitnc_plan_destroy(mitnc_plan* plan);
void mitnc_network_destroy(mitnc_network* net);
/* Message of the last failing call on this thread ("" if none); valid until
 * the next failing call on the same thread. */
const char* mitnc_last_error(void);

/* Kernel class ids (mitnc_plan_stats.steps_by_class index, force_kernel). */
enum {
  MITNC_K_SMALL = 0,  /* tiny step: one thread per output entry */
  MITNC_K_STEM = 1,   /* big tensor times small matrix: vector FMA, one thread per row */
  MITNC_K_TILE = 2,   /* LDS-staged, bit-permuted tiles, complex GEMM on FP32 MFMA */
  MITNC_K_TALL = 3,   /* as TILE with a 128 x 16 tile for narrow N */
  MITNC_K_SPLITK = 4, /* small M, N, long K: K split over workgroups, FP64 reduction;
                         complex64 steps with M N <= 16 per batch index and
                         K >= 2^8 run on a register-only kernel (one wave per
                         k split and batch index), the others on LDS tiles */
  MITNC_K_STREAM = 5  /* big tensor times small matrix on MFMA, streamed with no LDS staging:
                         needs at most 2^10 batch indices, M >= 2^8, K <= 64, N <= 64,
                         max(K/4, 1) * max(N/16, 1) <= 16, and the row indices
                         past the lowest four of A in the same relative order
                         in C (the planner's own output layouts satisfy this) */
};

#ifdef __cplusplus
}
#endif
#endif
