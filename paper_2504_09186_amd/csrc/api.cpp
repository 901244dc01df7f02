// extern "C" entry points of libmitnc (declared in include/mitnc.h) and the
// slice executor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <thread>

#include "kernels.hpp"
#include "plan.hpp"

using namespace mitnc;

static thread_local std::string g_err;

template <class F>
static int32_t guarded(F&& f) {
  try {
    f();
    return MITNC_OK;
  } catch (const Error& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host out of memory";
    return MITNC_INVALID_ARG;
  } catch (const std::exception& e) {
    g_err = e.what();
    return MITNC_INVALID_ARG;
  }
}

static void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(MITNC_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
}

// Slice ranges of plans with merged bits cover whole merge groups.
static void check_range(const mitnc_plan* P, uint64_t s0, uint64_t s1) {
  const uint64_t n_slices = 1ull << P->S;
  if (s0 >= s1 || s1 > n_slices) fail(MITNC_INVALID_ARG, "slice range out of bounds");
  const uint64_t am = (1ull << P->merge_align_bits) - 1;
  if ((s0 & am) || (s1 & am))
    fail(MITNC_INVALID_ARG, "slice range must be a multiple of 2^" + std::to_string(P->merge_align_bits) +
                                " (merged slice-id bits)");
  const int pw = P->opts.prologue_bits;
  if (pw > 0 && (s0 >> pw) != ((s1 - 1) >> pw))
    fail(MITNC_INVALID_ARG, "slice range must lie in one aligned block of 2^" + std::to_string(pw) +
                                " slices (prologue_bits)");
}

// Calls f(slice, step, mode) for every launch of slices s0 .. s1-1, in order
// (mode 1: store / accumulate at the root, 2: merge term).  The steps of the
// range prologue come first (level by level, at slice s0), or not at all
// with list_prologue false (the caller launches them batched).
template <class F>
static void for_each_launch(const mitnc_plan* P, uint64_t s0, uint64_t s1, F&& f, bool list_prologue = true) {
  SliceSchedule sched(P->nodes.size());
  if (list_prologue)
    for (int i : P->prologue_order) f(s0, (size_t)i, 1);
  for (uint64_t sl = s0; sl < s1; ++sl)
    for (size_t i = 0; i < P->steps.size(); ++i) {
      const PlanNode& O = P->nodes[P->steps[i].out];
      const int mode = sched.decide(P->steps[i].out, O.elig, O.emask, O.bmask, sl);
      if (mode && P->fwd_run_of[i] < 0) f(sl, i, P->steps[i].root ? 1 : mode);
    }
}

extern "C" {

const char* mitnc_last_error(void) { return g_err.c_str(); }

int32_t mitnc_network_from_circuit(int32_t n_qubits, int32_t n_gates, const mitnc_gate* gates,
                                   mitnc_network** out) {
  return guarded([&] {
    if (!out || n_qubits <= 0 || n_qubits > 65535 || n_gates < 0 || (n_gates > 0 && !gates))
      fail(MITNC_INVALID_ARG, "bad arguments");
    auto net = std::make_unique<mitnc_network>();
    net->n_qubits = n_qubits;
    std::vector<int32_t> seg(n_qubits, 0);
    for (int g = 0; g < n_gates; ++g) {
      const mitnc_gate& G = gates[g];
      if (!G.mat) fail(MITNC_INVALID_ARG, "gate matrix is null");
      Leaf L;
      L.gate = g;
      L.arity = G.arity;
      if (G.arity == 1) {
        if (G.q0 < 0 || G.q0 >= n_qubits) fail(MITNC_INVALID_ARG, "gate qubit out of range");
        int q = G.q0;
        int64_t lin = wire_label(q, seg[q]);
        int64_t lout = wire_label(q, ++seg[q]);
        // U[out][in] row-major: address bit 0 = in, bit 1 = out.
        L.labels = {lin, lout};
        L.data.resize(4);
        for (int e = 0; e < 4; ++e) L.data[e] = cd(G.mat[2 * e], G.mat[2 * e + 1]);
      } else if (G.arity == 2) {
        int q0 = G.q0, q1 = G.q1;
        if (q0 < 0 || q1 < 0 || q0 >= n_qubits || q1 >= n_qubits || q0 == q1)
          fail(MITNC_INVALID_ARG, "two-qubit gate qubits invalid");
        int64_t i0 = wire_label(q0, seg[q0]), i1 = wire_label(q1, seg[q1]);
        int64_t o0 = wire_label(q0, ++seg[q0]), o1 = wire_label(q1, ++seg[q1]);
        // U[o0 o1][i0 i1] row-major: bits (LSB first) i1, i0, o1, o0.
        L.labels = {i1, i0, o1, o0};
        L.data.resize(16);
        for (int e = 0; e < 16; ++e) L.data[e] = cd(G.mat[2 * e], G.mat[2 * e + 1]);
      } else {
        fail(MITNC_INVALID_ARG, "gate arity must be 1 or 2");
      }
      net->leaves.push_back(std::move(L));
    }
    for (int q = 0; q < n_qubits; ++q) {
      Leaf L;
      L.labels = {wire_label(q, 0)};
      L.data = {cd(1, 0), cd(0, 0)};
      net->leaves.push_back(std::move(L));
    }
    net->segs = seg;
    *out = net.release();
  });
}

int32_t mitnc_network_set_output(mitnc_network* net, const int8_t* per_qubit, int32_t n_batch,
                                 const uint8_t* batch_bits) {
  return guarded([&] {
    if (!net || !per_qubit) fail(MITNC_INVALID_ARG, "null argument");
    if (net->output_set) fail(MITNC_INVALID_ARG, "output already set");
    int n = net->n_qubits;
    std::vector<int> batched;
    for (int q = 0; q < n; ++q) {
      int v = per_qubit[q];
      if (v < -2 || v > 1) fail(MITNC_INVALID_ARG, "output spec must be 0, 1, -1 or -2");
      if (v == -2) batched.push_back(q);
    }
    int nbb = 0;
    if (!batched.empty()) {
      if (n_batch < 1 || (n_batch & (n_batch - 1)) || !batch_bits)
        fail(MITNC_INVALID_ARG, "n_batch must be a power of two and batch_bits given");
      while ((1 << nbb) < n_batch) ++nbb;
    }
    net->n_batch_bits = nbb;
    for (int q = 0; q < n; ++q) {
      int v = per_qubit[q];
      int64_t last = wire_label(q, net->segs[q]);
      if (v == 0 || v == 1) {
        Leaf L;
        L.labels = {last};
        L.data = {cd(v == 0 ? 1 : 0, 0), cd(v == 1 ? 1 : 0, 0)};
        net->leaves.push_back(std::move(L));
      } else if (v == -2) {
        int col = (int)(std::find(batched.begin(), batched.end(), q) - batched.begin());
        Leaf L;
        L.labels = {last};
        for (int j = 0; j < nbb; ++j) L.labels.push_back(batch_label(j));
        L.data.assign((size_t)2 << nbb, cd(0, 0));
        for (int b = 0; b < n_batch; ++b) {
          int x = batch_bits[(size_t)b * batched.size() + col] ? 1 : 0;
          L.data[(size_t)b * 2 + x] = cd(1, 0);
        }
        net->leaves.push_back(std::move(L));
      }
    }
    // Result layout (LSB first): open qubits from the highest to the lowest
    // qubit, then the batch bits.
    for (int q = n - 1; q >= 0; --q)
      if (per_qubit[q] == -1) net->output_lsb.push_back(wire_label(q, net->segs[q]));
    for (int j = 0; j < nbb; ++j) net->output_lsb.push_back(batch_label(j));
    net->output_set = true;
  });
}

int32_t mitnc_network_info(const mitnc_network* net, int32_t* n_leaves, int32_t* n_labels) {
  return guarded([&] {
    if (!net) fail(MITNC_INVALID_ARG, "null network");
    if (n_leaves) *n_leaves = (int32_t)net->leaves.size();
    if (n_labels) *n_labels = make_symnet(net->leaves, net->output_lsb).n_labels;
  });
}

static std::vector<int> dense_sliced(const SymNet& sn, const std::vector<int64_t>& ids) {
  std::vector<int> v;
  for (auto x : ids) v.push_back(sn.dense.at(x));
  return v;
}

int32_t mitnc_path_search(mitnc_network* net, const mitnc_search_opts* o) {
  return guarded([&] {
    if (!net || !o) fail(MITNC_INVALID_ARG, "null argument");
    if (!net->output_set) fail(MITNC_INVALID_ARG, "output not set");
    SymNet sn = make_symnet(net->leaves, net->output_lsb);
    int trials = std::max(1, o->trials);
    std::mt19937_64 rng(o->seed);
    const double alphas[] = {1.0, 0.5, 1.5, 2.0};
    const double temps[] = {0.02, 0.05, 0.1, 0.2};
    // With keep_slicing the current sliced indices are fixed: paths are
    // searched on the network without them, and further indices are sliced
    // only if the size cap requires it.
    std::vector<char> fixed(sn.n_labels, 0);
    std::vector<int> fixed_list;
    if (o->keep_slicing)
      for (auto x : net->sliced) {
        fixed[sn.dense.at(x)] = 1;
        fixed_list.push_back(sn.dense.at(x));
      }
    double best = -1;
    Path best_path;
    std::vector<int> best_sl;
    const int method = o->method;
    if (method < 0 || method > 2) fail(MITNC_INVALID_ARG, "unknown search method");
    if (o->window_bits < 0 || o->window_bits > 62) fail(MITNC_INVALID_ARG, "window_bits out of range");
    if (o->merge_bits < 0 || o->merge_bits > 12) fail(MITNC_INVALID_ARG, "merge_bits out of range (0..12)");
    if (!(o->launch_cost_flops >= 0)) fail(MITNC_INVALID_ARG, "launch_cost_flops must be >= 0");
    const double imbs[] = {0.05, 0.1, 0.2, 0.3, 0.5};
    const int cutoffs[] = {4, 6, 8, 10, 12};
    const double exts[] = {0.0, 0.25, 0.5, 1.0};
    std::vector<char> none(sn.n_labels, 0);
    const std::vector<char>& rm = o->keep_slicing ? fixed : none;
    const int n_runs = method == 2 ? 2 * trials : trials;
    // Parameters of every run are drawn first, in run order, so that the
    // runs can go in parallel and the result does not depend on the thread
    // count; ties keep the earliest run.
    struct Run {
      bool bisect;
      double alpha, tau;
      PartitionParams prm;
      uint64_t seed;
      double f = -1;
      Path path;
      std::vector<int> sl;
    };
    std::vector<Run> runs(n_runs);
    for (int r = 0; r < n_runs; ++r) {
      Run& R = runs[r];
      R.bisect = method == 1 || (method == 2 && r >= trials);
      const int t = method == 2 ? r % trials : r;
      if (R.bisect) {
        R.prm.imbalance = imbs[rng() % 5];
        R.prm.cutoff = cutoffs[rng() % 5];
        R.prm.ext_weight = exts[rng() % 4];
        R.prm.starts = 4;
        R.seed = rng();
      } else {
        R.alpha = t == 0 ? 1.0 : alphas[rng() % 4];
        R.tau = t == 0 ? 0.0 : temps[rng() % 4];
        R.seed = rng();
      }
    }
    auto run_one = [&](Run& R) {
      const bool bisect = R.bisect;
      Path p = bisect ? partition_path(sn, rm, R.prm, R.seed)
                      : greedy_path(sn, R.alpha, R.tau, R.seed, o->keep_slicing ? &fixed : nullptr);
      {
        // local refinement before slicing: no intermediate may grow
        const int width = sym_max_bits(sn, sym_run(sn, p, rm), rm);
        p = optimize_path(sn, p, &rm, width, 4);
      }
      bool ok;
      std::vector<int> sl;
      if (bisect) {
        // slicing interleaved with re-optimisation of the tree
        std::vector<int> extra = slice_reconf(sn, p, fixed_list, o->max_log2_elems, o->min_sliced, o->max_sliced, 2, &ok);
        sl = fixed_list;
        sl.insert(sl.end(), extra.begin(), extra.end());
      } else if (o->keep_slicing) {
        SymNet sub = sn;
        for (auto& v : sub.leaf) {
          std::vector<int> w;
          for (int x : v)
            if (!fixed[x]) w.push_back(x);
          v.swap(w);
        }
        for (int x : fixed_list) sub.closed[x] = 0;
        int extra_min = std::max(0, o->min_sliced - (int)fixed_list.size());
        int extra_max = std::max(0, o->max_sliced - (int)fixed_list.size());
        std::vector<int> extra = greedy_slices(sub, p, o->max_log2_elems, extra_min, extra_max, &ok);
        sl = fixed_list;
        sl.insert(sl.end(), extra.begin(), extra.end());
      } else {
        sl = greedy_slices(sn, p, o->max_log2_elems, o->min_sliced, o->max_sliced, &ok);
      }
      if (!ok) return;
      std::vector<char> m(sn.n_labels, 0);
      for (int x : sl) m[x] = 1;
      // refine again for the per-slice network, keeping the size cap
      p = optimize_path(sn, p, &m, std::max(o->max_log2_elems, sym_max_bits(sn, sym_run(sn, p, m), m)), 4);
      // Method 0 ranks by the flops of all slices; methods 1 and 2 rank every
      // trial by the flops executed with shared-prefix reuse (Sec. III-B),
      // sliced indices in the order the plan will use, over all slices or
      // over one aligned window of 2^window_bits slices.
      double f;
      if (method != 0) {
        std::vector<int> extra(sl.begin() + fixed_list.size(), sl.end());
        std::vector<int> ord = fixed_list;
        for (int x : order_slices(sn, p, extra)) ord.push_back(x);
        f = reuse_total_flops(sn, p, ord, o->window_bits, o->merge_bits, o->launch_cost_flops);
      } else {
        f = sym_total_flops(sym_run(sn, p, m)) * std::ldexp(1.0, (int)sl.size());
      }
      R.f = f;
      R.path = std::move(p);
      R.sl = std::move(sl);
    };
    {
      const int nth = std::max(1, std::min<int>(n_runs, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
      std::atomic<int> next{0};
      std::vector<std::thread> pool;
      std::vector<std::string> errs(nth);
      for (int i = 0; i < nth; ++i)
        pool.emplace_back([&, i] {
          try {
            for (int r; (r = next.fetch_add(1)) < n_runs;) run_one(runs[r]);
          } catch (const Error& e) {
            errs[i] = e.msg;
          } catch (const std::exception& e) {
            errs[i] = e.what();
          }
        });
      for (auto& th : pool) th.join();
      for (auto& e : errs)
        if (!e.empty()) fail(MITNC_INVALID_ARG, "path search: " + e);
    }
    for (Run& R : runs) {
      if (R.f < 0) continue;
      if (best < 0 || R.f < best) {
        best = R.f;
        best_path = R.path;
        best_sl = R.sl;
      }
    }
    if (best < 0) fail(MITNC_UNSUPPORTED, "no path met the size cap within max_sliced");
    net->path = best_path;
    net->sliced.clear();
    if (o->keep_slicing) {
      // the given indices keep their order (outer); added ones go inside
      std::vector<int> extra(best_sl.begin() + fixed_list.size(), best_sl.end());
      for (int x : fixed_list) net->sliced.push_back(sn.label_id[x]);
      for (int x : order_slices(sn, best_path, extra)) net->sliced.push_back(sn.label_id[x]);
    } else {
      for (int x : order_slices(sn, best_path, best_sl)) net->sliced.push_back(sn.label_id[x]);
    }
    if (o->branch_exchange) {
      std::vector<int> ord;
      for (auto x : net->sliced) ord.push_back(sn.dense.at(x));
      std::vector<char> m(sn.n_labels, 0);
      for (int x : ord) m[x] = 1;
      const int cap = std::max<int>(o->max_log2_elems, sym_max_bits(sn, sym_run(sn, net->path, m), m));
      net->path = branch_exchange(sn, net->path, ord, o->window_bits, o->merge_bits, cap, 8, nullptr, nullptr,
                                  o->launch_cost_flops);
    }
  });
}

int32_t mitnc_get_path(const mitnc_network* net, int32_t* pairs_out) {
  return guarded([&] {
    if (!net || !pairs_out) fail(MITNC_INVALID_ARG, "null argument");
    if (net->path.empty()) fail(MITNC_PATH_INVALID, "no path");
    for (size_t s = 0; s < net->path.size(); ++s) {
      pairs_out[2 * s] = net->path[s].first;
      pairs_out[2 * s + 1] = net->path[s].second;
    }
  });
}

int32_t mitnc_set_path(mitnc_network* net, int32_t n_steps, const int32_t* pairs) {
  return guarded([&] {
    if (!net || !pairs) fail(MITNC_INVALID_ARG, "null argument");
    Path p;
    for (int s = 0; s < n_steps; ++s) p.push_back({pairs[2 * s], pairs[2 * s + 1]});
    validate_path((int)net->leaves.size(), p);
    net->path = p;
  });
}

int32_t mitnc_get_slicing(const mitnc_network* net, int32_t* n_out, int64_t* ids_out) {
  return guarded([&] {
    if (!net || !n_out) fail(MITNC_INVALID_ARG, "null argument");
    *n_out = (int32_t)net->sliced.size();
    if (ids_out)
      for (size_t i = 0; i < net->sliced.size(); ++i) ids_out[i] = net->sliced[i];
  });
}

int32_t mitnc_set_slicing(mitnc_network* net, int32_t n, const int64_t* ids) {
  return guarded([&] {
    if (!net || n < 0 || n > 62 || (n > 0 && !ids)) fail(MITNC_INVALID_ARG, "bad arguments");
    if (!net->output_set) fail(MITNC_INVALID_ARG, "output not set");
    SymNet sn = make_symnet(net->leaves, net->output_lsb);
    std::vector<int64_t> v;
    for (int i = 0; i < n; ++i) {
      auto it = sn.dense.find(ids[i]);
      if (it == sn.dense.end() || !sn.closed[it->second])
        fail(MITNC_INVALID_ARG, "label " + std::to_string(ids[i]) + " is not a closed edge");
      if (std::find(v.begin(), v.end(), ids[i]) != v.end()) fail(MITNC_INVALID_ARG, "duplicate sliced label");
      v.push_back(ids[i]);
    }
    net->sliced = v;
  });
}

int32_t mitnc_slice_greedy(mitnc_network* net, int32_t max_log2_elems, int32_t min_sliced, int32_t max_sliced,
                           int32_t* n_out, int64_t* ids_out) {
  return guarded([&] {
    if (!net) fail(MITNC_INVALID_ARG, "null network");
    if (net->path.empty()) fail(MITNC_PATH_INVALID, "no path");
    if (max_sliced > 64) fail(MITNC_INVALID_ARG, "at most 64 sliced indices");
    SymNet sn = make_symnet(net->leaves, net->output_lsb);
    bool ok;
    auto sl = greedy_slices(sn, net->path, max_log2_elems, min_sliced, max_sliced, &ok);
    if (!ok) fail(MITNC_UNSUPPORTED, "cap not met within max_sliced");
    net->sliced.clear();
    for (int x : order_slices(sn, net->path, sl)) net->sliced.push_back(sn.label_id[x]);
    if (n_out) *n_out = (int32_t)net->sliced.size();
    if (ids_out)
      for (size_t i = 0; i < net->sliced.size(); ++i) ids_out[i] = net->sliced[i];
  });
}

int32_t mitnc_branch_exchange(mitnc_network* net, int32_t window_bits, int32_t merge_bits, int32_t max_log2_elems,
                              int32_t passes, double launch_cost_flops, double* flops_before, double* flops_after) {
  return guarded([&] {
    if (!net) fail(MITNC_INVALID_ARG, "null network");
    if (net->path.empty()) fail(MITNC_INVALID_ARG, "no path");
    if (window_bits < 0 || window_bits > 62 || merge_bits < 0 || merge_bits > 12 || passes < 0 || max_log2_elems < 0 ||
        !(launch_cost_flops >= 0))
      fail(MITNC_INVALID_ARG, "bad argument");
    SymNet sn = make_symnet(net->leaves, net->output_lsb);
    std::vector<int> ord;
    for (auto x : net->sliced) ord.push_back(sn.dense.at(x));
    double b = 0, a = 0;
    net->path = branch_exchange(sn, net->path, ord, window_bits, merge_bits, max_log2_elems, passes, &b, &a,
                                launch_cost_flops);
    if (flops_before) *flops_before = b;
    if (flops_after) *flops_after = a;
  });
}

int32_t mitnc_index_overhead(const mitnc_network* net, int64_t label, double* overhead) {
  return guarded([&] {
    if (!net || !overhead) fail(MITNC_INVALID_ARG, "null argument");
    if (net->path.empty()) fail(MITNC_PATH_INVALID, "no path");
    SymNet sn = make_symnet(net->leaves, net->output_lsb);
    auto it = sn.dense.find(label);
    if (it == sn.dense.end() || !sn.closed[it->second]) fail(MITNC_INVALID_ARG, "label is not a closed edge");
    std::vector<char> m(sn.n_labels, 0);
    for (int x : dense_sliced(sn, net->sliced)) m[x] = 1;
    double c_ori = sym_total_flops(sym_run(sn, net->path, m));
    m[it->second] = 1;
    double c_a = sym_total_flops(sym_run(sn, net->path, m));
    *overhead = 2.0 * c_a / c_ori;
  });
}

int32_t mitnc_plan_create(const mitnc_network* net, const mitnc_plan_opts* opts, mitnc_plan** out) {
  return guarded([&] {
    if (!net || !opts || !out) fail(MITNC_INVALID_ARG, "null argument");
    *out = build_plan(net, *opts);
  });
}

int32_t mitnc_plan_query(const mitnc_plan* P, mitnc_plan_stats* st) {
  return guarded([&] {
    if (!P || !st) fail(MITNC_INVALID_ARG, "null argument");
    std::memset(st, 0, sizeof(*st));
    st->workspace_bytes = P->ws_bytes;
    st->result_elems = P->result_elems;
    st->n_sliced = P->S;
    st->n_steps = (int32_t)P->steps.size();
    st->max_log2_elems = P->max_log2;
    st->n_kernel_classes = 6;
    double nsl = std::ldexp(1.0, P->S);
    for (auto& s : P->steps) {
      st->flops_full_slice += s.flops_slice;
      st->bytes_full_slice += s.bytes_slice;
      st->steps_by_class[s.kclass] += 1;
      st->flops_by_class[s.kclass] += s.flops_slice;
      // how many of the 2^S slices (run in order from 0) compute this step
      const PlanNode& O = P->nodes[s.out];
      double runs = std::min(merge_runs(O.elig, O.emask, O.bmask, P->S, P->S), nsl);
      st->flops_reused_slice += s.flops * runs / nsl;
      st->bytes_reused_slice += s.bytes * runs / nsl;
    }
    st->n_merged = __builtin_popcountll(P->merged);
    st->merge_align_bits = P->merge_align_bits;
    st->merged_mask = P->merged;
    st->n_reverse_groups = P->rev_groups.empty() ? 0 : (int32_t)P->rev_groups.size() - 1;
    st->n_batched_small = (int32_t)P->prologue_order.size();
    for (const mitnc_plan::FwdRun& R : P->fwd_runs) st->n_batched_launches += (int32_t)R.levels.size();
    st->n_grad_gates = P->n_grad_gates;
    st->n_reverse_ops = (int32_t)P->rev.size();
    st->flops_reverse_slice = P->rev_flops;
  });
}

int32_t mitnc_plan_steps(const mitnc_plan* P, double* info) {
  return guarded([&] {
    if (!P || !info) fail(MITNC_INVALID_ARG, "null argument");
    for (size_t i = 0; i < P->steps.size(); ++i) {
      const PlanStep& s = P->steps[i];
      double* r = info + 12 * i;
      int lo = P->nodes[s.out].lo;
      r[0] = s.kclass;
      r[1] = s.d.mb;
      r[2] = s.d.nb;
      r[3] = s.d.kb;
      r[4] = s.d.bb;
      r[5] = lo >= kLevelNever ? -1 : lo;
      r[6] = s.flops;
      r[7] = s.bytes;
      r[8] = std::ldexp(1.0, s.d.ks_bits);
      r[9] = s.swapped;
      r[10] = P->nodes[s.out].rank;
      r[11] = s.root;
    }
  });
}

int32_t mitnc_plan_step_info(const mitnc_plan* P, int32_t step, mitnc_step_info* info) {
  return guarded([&] {
    if (!P || !info) fail(MITNC_INVALID_ARG, "null argument");
    if (step < 0 || step >= (int32_t)P->steps.size()) fail(MITNC_INVALID_ARG, "step out of range");
    const PlanStep& s = P->steps[step];
    const StepDesc& d = s.d;
    std::memset(info, 0, sizeof(*info));
    info->a = s.a;
    info->b = s.b;
    info->out = s.out;
    info->root = s.root;
    info->kernel_class = s.kclass;
    info->section = P->step_section.empty() ? -1 : P->step_section[step];
    info->section_pos = info->section_len = 0;
    if (info->section >= 0) {
      const auto& m = P->sections[info->section].steps;
      info->section_len = (int32_t)m.size();
      info->section_pos = (int32_t)(std::find(m.begin(), m.end(), step) - m.begin());
    }
    info->mb = d.mb;
    info->nb = d.nb;
    info->kb = d.kb;
    info->bb = d.bb;
    std::memcpy(info->am, d.am, 32);
    std::memcpy(info->ak, d.ak, 32);
    std::memcpy(info->ab, d.ab, 32);
    std::memcpy(info->bk, d.bk, 32);
    std::memcpy(info->bn, d.bn, 32);
    std::memcpy(info->bbt, d.bbt, 32);
    std::memcpy(info->cm, d.cm, 32);
    std::memcpy(info->cn, d.cn, 32);
    std::memcpy(info->cb, d.cb, 32);
    if (s.kclass == MITNC_K_TILE || s.kclass == MITNC_K_TALL || s.kclass == MITNC_K_SPLITK) {
      info->tm = d.tm;
      info->tn = d.tn;
      info->tk = d.tk;
      std::memcpy(info->a_tile, d.a_tile, 16);
      std::memcpy(info->b_tile, d.b_tile, 16);
      std::memcpy(info->lds_a_swz, d.a_swz, 8);
      std::memcpy(info->lds_b_swz, d.b_swz, 8);
      std::memcpy(info->lds_a_row, d.ha_row, sizeof d.ha_row);
      std::memcpy(info->lds_b_row, d.hb_row, sizeof d.hb_row);
      std::memcpy(info->lds_k_col, d.hk, 8);
      info->vec_a = d.vec_a;
      info->vec_b = d.vec_b;
    }
  });
}

int32_t mitnc_plan_reverse_info(const mitnc_plan* P, int32_t op, mitnc_step_info* info, int32_t* n_ops) {
  return guarded([&] {
    if (!P || !n_ops) fail(MITNC_INVALID_ARG, "null argument");
    // Execution order: level by level, each level's MFMA-class ops, then its
    // SMALL ops in block-table order.
    std::vector<std::pair<int, int>> order;  // (rev index, level)
    for (size_t lv = 0; lv < P->rev_levels.size(); ++lv) {
      for (int ri : P->rev_levels[lv].big) order.push_back({ri, (int)lv});
      for (size_t i = 0; i < P->rev.size(); ++i)
        if (P->rev[i].kclass == MITNC_K_SMALL && P->rev_level_of[i] == (int)lv &&
            small_bounded(P->rev[i].d.mb, P->rev[i].d.nb, P->rev[i].d.kb, P->rev[i].d.bb))
          order.push_back({(int)i, (int)lv});
    }
    *n_ops = (int32_t)order.size();
    if (!info) return;
    if (op < 0 || op >= (int32_t)order.size()) fail(MITNC_INVALID_ARG, "reverse op out of range");
    const RevOp& r = P->rev[order[op].first];
    const StepDesc& d = r.d;
    std::memset(info, 0, sizeof(*info));
    info->a = P->steps[r.step].out;
    info->b = r.other;
    info->out = r.target;
    info->root = order[op].second;
    info->kernel_class = r.kclass;
    info->section = -1;
    info->mb = d.mb;
    info->nb = d.nb;
    info->kb = d.kb;
    info->bb = d.bb;
    std::memcpy(info->am, d.am, 32);
    std::memcpy(info->ak, d.ak, 32);
    std::memcpy(info->ab, d.ab, 32);
    std::memcpy(info->bk, d.bk, 32);
    std::memcpy(info->bn, d.bn, 32);
    std::memcpy(info->bbt, d.bbt, 32);
    std::memcpy(info->cm, d.cm, 32);
    std::memcpy(info->cn, d.cn, 32);
    std::memcpy(info->cb, d.cb, 32);
  });
}

int32_t mitnc_plan_node_info(const mitnc_plan* P, int32_t node, mitnc_node_info* info) {
  return guarded([&] {
    if (!P || !info) fail(MITNC_INVALID_ARG, "null argument");
    if (node < 0 || node >= (int32_t)P->nodes.size()) fail(MITNC_INVALID_ARG, "node out of range");
    const PlanNode& nd = P->nodes[node];
    std::memset(info, 0, sizeof(*info));
    info->is_leaf = nd.leaf;
    info->rank = nd.rank;
    info->full_rank = nd.full_rank;
    info->level = nd.lo >= kLevelNever ? -1 : nd.lo;
    info->hoisted = nd.hoisted;
    info->n_slice_bits = (int32_t)nd.slice_bits.size();
    for (size_t j = 0; j < nd.slice_bits.size() && j < 64; ++j) {
      info->slice_bit[j] = nd.slice_bits[j].first;
      info->slice_pos[j] = nd.slice_bits[j].second;
    }
    info->elig_mask = nd.elig;
    info->recompute_mask = nd.emask;
    info->merge_mask = nd.bmask;
    info->merge_tmp_offset = nd.bmask ? P->off_arena + nd.tmp_offset : 0;
    switch (nd.region) {
      case 0: info->ws_offset = nd.offset; break;
      case 1: info->ws_offset = P->off_persist + nd.offset; break;
      case 2: info->ws_offset = P->off_arena + nd.offset; break;
      default: info->ws_offset = UINT64_MAX;
    }
  });
}

int32_t mitnc_plan_leaf_data(const mitnc_plan* P, int32_t leaf, float* out, uint64_t capacity_floats,
                             uint64_t* n_floats) {
  return guarded([&] {
    if (!P || !n_floats) fail(MITNC_INVALID_ARG, "null argument");
    if (leaf < 0 || leaf >= P->n_leaves) fail(MITNC_INVALID_ARG, "leaf out of range");
    const auto& v = P->leaf_data[leaf];
    *n_floats = v.size();
    if (out) {
      if (capacity_floats < v.size()) fail(MITNC_INVALID_ARG, "output buffer too small");
      std::memcpy(out, v.data(), v.size() * sizeof(float));
    }
  });
}

int32_t mitnc_plan_upload(mitnc_plan* P, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    if (!P || !ws) fail(MITNC_INVALID_ARG, "null argument");
    if (ws_bytes < P->ws_bytes) fail(MITNC_WORKSPACE_TOO_SMALL, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    if (P->opts.precision != MITNC_C64) P->calibrated = false;
    for (int i = 0; i < P->n_leaves; ++i) {
      const auto& h = P->leaf_data[i];
      hip_check(hipMemcpyAsync(base + P->nodes[i].offset, h.data(), h.size() * sizeof(float),
                               hipMemcpyHostToDevice, s),
                "leaf upload");
      if (!P->leaf_half.empty()) {
        const auto& w = P->leaf_half[i];
        hip_check(hipMemcpyAsync(base + P->off_leaf_half + P->nodes[i].offset / 2, w.data(),
                                 w.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s),
                  "leaf upload");
      }
    }
    hip_check(hipMemsetAsync(base + P->off_stats, 0, 4 * P->steps.size(), s), "stats reset");
    if (!P->gtab.empty())
      hip_check(hipMemcpyAsync(base + P->off_gtab, P->gtab.data(), sizeof(GradEntry) * P->gtab.size(),
                               hipMemcpyHostToDevice, s),
                "gradient table upload");
    if (!P->rtab.empty()) {
      hip_check(hipMemcpyAsync(base + P->off_rtab, P->rtab.data(), sizeof(SmallRevOp) * P->rtab.size(),
                               hipMemcpyHostToDevice, s),
                "reverse table upload");
      hip_check(hipMemcpyAsync(base + P->off_rblock, P->rblock.data(), sizeof(uint32_t) * P->rblock.size(),
                               hipMemcpyHostToDevice, s),
                "reverse block table upload");
    }
    auto put = [&](uint64_t off, const void* src, size_t bytes) {
      if (bytes) hip_check(hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s), "batch table upload");
    };
    put(P->off_ftab, P->ftab.data(), sizeof(SmallFwdOp) * P->ftab.size());
    put(P->off_fblock, P->fblock.data(), sizeof(uint32_t) * P->fblock.size());
    put(P->off_ftab64, P->ftab64.data(), sizeof(SmallFwdOp) * P->ftab64.size());
    put(P->off_fblock64, P->fblock64.data(), sizeof(uint32_t) * P->fblock64.size());
    hip_check(hipStreamSynchronize(s), "leaf upload sync");
    P->ftab_uploaded = P->ftab_version;
    P->uploaded = true;
    P->valid_slice = -1;
    P->uploaded_ws = ws;
  });
}

mitnc_plan::~mitnc_plan() {
  for (void* e : ev_pool) hipEventDestroy((hipEvent_t)e);
}

// Launches one step.  prec: storage precision of this run (the plan's own,
// or complex64 for a calibration slice of an FP16/BF16 plan).
static void launch_plan_step(mitnc_plan* P, PlanStep& st, char* base, uint64_t slice, double* acc,
                             hipStream_t s, int prec, bool stats, bool merge_term = false) {
  StepDesc d = (prec == MITNC_C64 && P->opts.precision != MITNC_C64) ? st.d64 : st.d;
  const bool half = prec != MITNC_C64;
  // Sliced leaves and hoisted results hold every value of their sliced
  // indices: a slice reads the sub-tensor at its own values (a hoisted step
  // writes the whole tensor).
  auto ptr = [&](int node, bool operand) -> char* {
    const PlanNode& nd = P->nodes[node];
    uint64_t e = 0;
    if (operand)
      for (auto& [sb, pb] : nd.slice_bits) e += ((slice >> sb) & 1ull) << pb;
    const uint64_t esz = half ? 4 : 8;
    uint64_t off;
    if (nd.region == 0) {
      off = half ? P->off_leaf_half + nd.offset / 2 : nd.offset;
    } else if (nd.region == 1) {
      off = P->off_persist + nd.offset;
    } else {
      off = P->off_arena + nd.offset;
    }
    return base + off + e * esz;
  };
  d.A = ptr(st.a, true);
  d.B = ptr(st.b, true);
  d.prec = prec;
  if (!half) {
    d.out_scale = 1.f;
    d.acc_scale = 1.0;
  }
  if (st.root) {
    d.C = nullptr;
    d.acc = acc;
    d.mode = EPI_ACC64;
  } else {
    // A merge term goes to the node's term buffer; it is then added.
    d.C = merge_term ? base + P->off_arena + P->nodes[st.out].tmp_offset : ptr(st.out, false);
    d.acc = nullptr;
    d.mode = EPI_STORE;
  }
  d.part = (float*)(base + P->off_part);
  d.stats = stats ? (float*)(base + P->off_stats) : nullptr;
  d.step_index = (int32_t)(&st - P->steps.data());
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (P->timing) {
    size_t need = 2 * (P->ev_used + 1);
    while (P->ev_pool.size() < need) {
      hipEvent_t e;
      hip_check(hipEventCreate(&e), "event create");
      P->ev_pool.push_back((void*)e);
    }
    e0 = (hipEvent_t)P->ev_pool[2 * P->ev_used];
    e1 = (hipEvent_t)P->ev_pool[2 * P->ev_used + 1];
    P->ev_step.push_back((int)(&st - P->steps.data()));
    P->ev_used++;
  }
  hip_check(launch_step(st.kclass, d, s, e0, e1), "kernel launch");
  if (merge_term) {
    if (P->timing) {
      while (P->ev_pool.size() < 2 * (P->ev_used + 1)) {
        hipEvent_t e;
        hip_check(hipEventCreate(&e), "event create");
        P->ev_pool.push_back((void*)e);
      }
      e0 = (hipEvent_t)P->ev_pool[2 * P->ev_used];
      e1 = (hipEvent_t)P->ev_pool[2 * P->ev_used + 1];
      P->ev_step.push_back(kMergeEvent - (4 * d.step_index + prec));
      P->ev_used++;
    }
    unsigned int* slot = stats ? (unsigned int*)(base + P->off_stats) + d.step_index : nullptr;
    hip_check(launch_merge_add(prec, ptr(st.out, false), d.C, 1ull << P->nodes[st.out].full_rank, slot, s, e0, e1),
              "merge add launch");
  }
}

// Launches a fused section (at the position of its last step).
static void launch_plan_section(mitnc_plan* P, PlanSection& sec, char* base, uint64_t slice, hipStream_t s,
                                int prec, bool stats) {
  const bool half = prec != MITNC_C64;
  auto ptr = [&](int node, bool operand) -> char* {
    const PlanNode& nd = P->nodes[node];
    uint64_t e = 0;
    if (operand)
      for (auto& [sb, pb] : nd.slice_bits) e += ((slice >> sb) & 1ull) << pb;
    uint64_t off = nd.region == 0 ? (half ? P->off_leaf_half + nd.offset / 2 : nd.offset)
                                  : (nd.region == 1 ? P->off_persist : P->off_arena) + nd.offset;
    return base + off + e * (half ? 4 : 8);
  };
  SectionDesc sd = sec.sd;
  sd.A = ptr(P->steps[sec.steps[0]].a, true);
  sd.C = ptr(P->steps[sec.steps.back()].out, false);
  sd.prec = prec;
  sd.stats = stats ? (float*)(base + P->off_stats) : nullptr;
  for (size_t j = 0; j < sec.steps.size(); ++j) {
    const PlanStep& st = P->steps[sec.steps[j]];
    sd.st[j].B = ptr(st.b, true);
    sd.st[j].out_scale = half ? st.d.out_scale : 1.f;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (P->timing) {
    size_t need = 2 * (P->ev_used + 1);
    while (P->ev_pool.size() < need) {
      hipEvent_t e;
      hip_check(hipEventCreate(&e), "event create");
      P->ev_pool.push_back((void*)e);
    }
    e0 = (hipEvent_t)P->ev_pool[2 * P->ev_used];
    e1 = (hipEvent_t)P->ev_pool[2 * P->ev_used + 1];
    P->ev_step.push_back(-1 - (int)(&sec - P->sections.data()));
    P->ev_used++;
  }
  hip_check(launch_section(sd, s, e0, e1), "section launch");
}

// One batched run of forward SMALL steps, level by level.  The table of the
// plan's precision carries each step's out_scale: it is copied again after
// the exponents change.
static void launch_fwd_run(mitnc_plan* P, int run, char* base, uint64_t slice, hipStream_t s, int prec, bool stats) {
  const bool c64_of_half = prec == MITNC_C64 && P->opts.precision != MITNC_C64;
  if (!c64_of_half && P->ftab_uploaded != P->ftab_version) {
    for (size_t e = 0; e < P->ftab.size(); ++e) P->ftab[e].d.out_scale = P->steps[P->ftab_step[e]].d.out_scale;
    if (P->opts.precision == MITNC_C64)
      for (auto& e : P->ftab) e.d.out_scale = 1.f;
    hip_check(hipMemcpyAsync(base + P->off_ftab, P->ftab.data(), sizeof(SmallFwdOp) * P->ftab.size(),
                             hipMemcpyHostToDevice, s),
              "batch table refresh");
    hip_check(hipStreamSynchronize(s), "batch table refresh sync");
    P->ftab_uploaded = P->ftab_version;
  }
  const mitnc_plan::FwdRun& R = P->fwd_runs[run];
  const auto& levels = c64_of_half ? R.levels64 : R.levels;
  const SmallFwdOp* tab = (const SmallFwdOp*)(base + (c64_of_half ? P->off_ftab64 : P->off_ftab));
  const uint32_t* blk = (const uint32_t*)(base + (c64_of_half ? P->off_fblock64 : P->off_fblock));
  for (size_t l = 0; l < levels.size(); ++l) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (P->timing) {
      while (P->ev_pool.size() < 2 * (P->ev_used + 1)) {
        hipEvent_t e;
        hip_check(hipEventCreate(&e), "event create");
        P->ev_pool.push_back((void*)e);
      }
      e0 = (hipEvent_t)P->ev_pool[2 * P->ev_used];
      e1 = (hipEvent_t)P->ev_pool[2 * P->ev_used + 1];
      P->ev_step.push_back(kFwdEvent - (int)l);
      P->ev_used++;
      hip_check(hipEventRecord(e0, s), "event record");
    }
    hip_check(launch_small_fwd(prec, tab, blk, levels[l].first, levels[l].blocks, base,
                               stats ? (float*)(base + P->off_stats) : nullptr, slice, s),
              "batched small launch");
    if (P->timing) hip_check(hipEventRecord(e1, s), "event record");
    // the level's other steps, one launch each
    for (int i : R.levels[l].big) launch_plan_step(P, P->steps[i], base, slice, nullptr, s, prec, stats);
  }
}

static void run_slices(mitnc_plan* P, char* base, uint64_t s0, uint64_t s1, double* acc, hipStream_t s, int prec,
                       bool stats) {
  if (!P->fwd_runs.empty()) launch_fwd_run(P, 0, base, s0, s, prec, stats);  // the range prologue
  for_each_launch(P, s0, s1, [&](uint64_t sl, size_t i, int mode) {
    PlanStep& st = P->steps[i];
    const int sec = P->step_section.empty() ? -1 : P->step_section[i];
    if (sec < 0) launch_plan_step(P, st, base, sl, acc, s, prec, stats, mode == 2);
    else if (P->sections[sec].steps.back() == (int)i) launch_plan_section(P, P->sections[sec], base, sl, s, prec, stats);
  }, false);
}

int32_t mitnc_plan_schedule(const mitnc_plan* P, uint64_t s0, uint64_t s1, int64_t capacity, int64_t* ops_out,
                            int64_t* n_ops) {
  return guarded([&] {
    if (!P || !n_ops || capacity < 0 || (capacity > 0 && !ops_out)) fail(MITNC_INVALID_ARG, "bad argument");
    check_range(P, s0, s1);
    int64_t k = 0;
    for_each_launch(P, s0, s1, [&](uint64_t sl, size_t i, int mode) {
      if (k < capacity) {
        ops_out[3 * k] = (int64_t)sl;
        ops_out[3 * k + 1] = (int64_t)i;
        ops_out[3 * k + 2] = mode;
      }
      ++k;
    });
    *n_ops = k;
  });
}

static void check_ws(mitnc_plan* P, void* ws, size_t ws_bytes) {
  if (!P || !ws) fail(MITNC_INVALID_ARG, "null argument");
  if (!P->uploaded || P->uploaded_ws != ws) fail(MITNC_INVALID_ARG, "plan not uploaded to this workspace");
  if (ws_bytes < P->ws_bytes) fail(MITNC_WORKSPACE_TOO_SMALL, "workspace too small");
}

// Exponents of an FP16/BF16 plan from complex64 maxima: runs slices s0 .. s1-1
// in complex64 (result into the calibration buffer), records each step's
// largest |Re|, |Im| and derives every tensor's exponent in path order;
// leaves the per-step maxima cleared.
static void calibrate_range(mitnc_plan* P, char* base, uint64_t s0, uint64_t s1, hipStream_t s) {
  const size_t nst = P->steps.size();
  hip_check(hipMemsetAsync(base + P->off_stats, 0, 4 * nst, s), "stats reset");
  hip_check(hipMemsetAsync(base + P->off_calib, 0, 16 * P->result_elems, s), "calibration result reset");
  run_slices(P, base, s0, s1, (double*)(base + P->off_calib), s, MITNC_C64, true);
  std::vector<float> mx(nst);
  hip_check(hipMemcpyAsync(mx.data(), base + P->off_stats, 4 * nst, hipMemcpyDeviceToHost, s), "stats read");
  hip_check(hipStreamSynchronize(s), "calibration sync");
  // Exponents in path order: stored C = true C * 2^-eC, and the kernel
  // result is (true A B) * 2^-(eA + eB).
  for (size_t i = 0; i < nst; ++i) {
    PlanStep& st = P->steps[i];
    const int ea = P->nodes[st.a].exp, eb = P->nodes[st.b].exp;
    if (st.root) {
      st.d.acc_scale = std::ldexp(1.0, ea + eb);
      st.d.out_scale = 1.f;
      continue;
    }
    // A step that was all zero in the calibration slices gets the exponent
    // of the worst case: |mantissa products| <= 2^14 * 2^14 per term, 2^kb
    // terms, so 2^(ea + eb + 14 + kb) keeps any later value below 2^14.
    const int ec = mx[i] > 0 ? mantissa_exponent((double)mx[i]) : ea + eb + 14 + st.d.kb;
    P->nodes[st.out].exp = ec;
    st.d.out_scale = (float)std::ldexp(1.0, ea + eb - ec);
    st.d.acc_scale = 1.0;
  }
  P->ftab_version++;
  hip_check(hipMemsetAsync(base + P->off_stats, 0, 4 * nst, s), "stats reset");
  P->calibrated = true;
}

// Checks the per-step maxima of the stored mantissas of one FP16/BF16 run:
// a value that is not finite or reaches the FP16 maximum (FP16 storage)
// overflowed; a largest value more than 2^4 away from the target range
// [2^13, 2^14) (below 2^9 or at or above 2^18) is an exponent miss.  Steps
// whose stored values were all zero carry no information and pass.
static bool maxima_ok(const mitnc_plan* P, const std::vector<float>& mx, int prec, std::string* why) {
  for (size_t i = 0; i < P->steps.size(); ++i) {
    if (P->steps[i].root) continue;
    const float m = mx[i];
    const bool over = !std::isfinite(m) || (prec == MITNC_CF16 && m >= 65504.f);
    const bool miss = m > 0.f && (m < 512.f || m >= 262144.f);
    if (over || miss) {
      if (why) *why = "step " + std::to_string(i) + (over ? ": overflow" : ": exponent miss") + " (largest stored " +
                      std::to_string(m) + ")";
      return false;
    }
  }
  return true;
}

int32_t mitnc_execute(mitnc_plan* P, void* ws, size_t ws_bytes, uint64_t s0, uint64_t s1, double* acc,
                      void* stream) {
  return guarded([&] {
    check_ws(P, ws, ws_bytes);
    if (!acc) fail(MITNC_INVALID_ARG, "null result");
    if (!P->calibrated) fail(MITNC_INVALID_ARG, "FP16/BF16 plan: call mitnc_calibrate first");
    check_range(P, s0, s1);
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    const int prec = P->opts.precision;
    if (prec == MITNC_C64) {
      run_slices(P, base, s0, s1, acc, s, prec, false);
      // every node of a differentiable plan now holds its value for s1 - 1
      P->valid_slice = P->opts.differentiable ? (int64_t)(s1 - 1) : -1;
      return;
    }
    // Precision form: the slices are summed into the calibration buffer and
    // added to the caller's result only once the stored maxima show no
    // overflow and no exponent miss; otherwise the exponents are re-derived
    // from complex64 maxima over this very slice range and the range runs
    // again (at most once; then MITNC_NUMERIC).
    const size_t nst = P->steps.size();
    double* stage = (double*)(base + P->off_calib);
    std::vector<float> mx(nst);
    std::string why;
    for (int attempt = 0;; ++attempt) {
      hip_check(hipMemsetAsync(base + P->off_stats, 0, 4 * nst, s), "stats reset");
      hip_check(hipMemsetAsync(stage, 0, 16 * P->result_elems, s), "staging reset");
      run_slices(P, base, s0, s1, stage, s, prec, true);
      hip_check(hipMemcpyAsync(mx.data(), base + P->off_stats, 4 * nst, hipMemcpyDeviceToHost, s), "stats read");
      hip_check(hipStreamSynchronize(s), "exponent check sync");
      if (maxima_ok(P, mx, prec, &why)) break;
      P->reruns++;
      if (attempt == 1 || P->opts.no_rerun)
        fail(MITNC_NUMERIC, "FP16/BF16 exponents: " + why + (P->opts.no_rerun ? " (re-run disabled)" : " after a re-run"));
      calibrate_range(P, base, s0, s1, s);
    }
    hip_check(launch_accumulate(acc, stage, P->result_elems, s), "result accumulate");
  });
}

int32_t mitnc_plan_exponents(mitnc_plan* P, int32_t* exps_out, const int32_t* exps_in, int32_t* reruns_out) {
  return guarded([&] {
    if (!P) fail(MITNC_INVALID_ARG, "null plan");
    if (exps_out)
      for (size_t i = 0; i < P->nodes.size(); ++i) exps_out[i] = P->nodes[i].exp;
    if (reruns_out) *reruns_out = P->reruns;
    if (!exps_in) return;
    if (P->opts.precision == MITNC_C64) fail(MITNC_INVALID_ARG, "complex64 plans have no exponents");
    for (size_t i = 0; i < P->steps.size(); ++i) {
      PlanStep& st = P->steps[i];
      if (!st.root) P->nodes[st.out].exp = exps_in[st.out];
    }
    for (size_t i = 0; i < P->steps.size(); ++i) {
      PlanStep& st = P->steps[i];
      const int ea = P->nodes[st.a].exp, eb = P->nodes[st.b].exp;
      if (st.root) {
        st.d.acc_scale = std::ldexp(1.0, ea + eb);
        st.d.out_scale = 1.f;
      } else {
        st.d.out_scale = (float)std::ldexp(1.0, ea + eb - P->nodes[st.out].exp);
        st.d.acc_scale = 1.0;
      }
    }
    P->ftab_version++;
  });
}

int32_t mitnc_calibrate(mitnc_plan* P, void* ws, size_t ws_bytes, uint64_t s0, uint64_t s1, void* stream) {
  return guarded([&] {
    check_ws(P, ws, ws_bytes);
    if (P->opts.precision == MITNC_C64) return;  // nothing to calibrate
    uint64_t n_slices = 1ull << P->S;
    if (s0 >= s1 || s1 > n_slices) fail(MITNC_INVALID_ARG, "slice range out of bounds");
    // with merged bits: the whole merge groups that hold the range
    const uint64_t am = (1ull << P->merge_align_bits) - 1;
    check_range(P, s0 & ~am, (s1 + am) & ~am);
    calibrate_range(P, (char*)ws, s0 & ~am, (s1 + am) & ~am, (hipStream_t)stream);
  });
}

int32_t mitnc_step_maxima(mitnc_plan* P, void* ws, size_t ws_bytes, float* out, int32_t reset, void* stream) {
  return guarded([&] {
    check_ws(P, ws, ws_bytes);
    if (!out) fail(MITNC_INVALID_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    const size_t nst = P->steps.size();
    hip_check(hipMemcpyAsync(out, base + P->off_stats, 4 * nst, hipMemcpyDeviceToHost, s), "stats read");
    hip_check(hipStreamSynchronize(s), "stats sync");
    if (reset) hip_check(hipMemsetAsync(base + P->off_stats, 0, 4 * nst, s), "stats reset");
  });
}

static char* node_value_ptr(mitnc_plan* P, char* base, int node, uint64_t slice) {
  const PlanNode& nd = P->nodes[node];
  if (nd.region == 0) {
    uint64_t e = 0;
    for (auto& [sb, pb] : nd.slice_bits) e += ((slice >> sb) & 1ull) << pb;
    return base + nd.offset + e * 8;
  }
  return base + (nd.region == 1 ? P->off_persist : P->off_arena) + nd.offset;
}

int32_t mitnc_backward(mitnc_plan* P, void* ws, size_t ws_bytes, uint64_t s0, uint64_t s1, const double* w,
                       double* grad, void* stream) {
  return guarded([&] {
    check_ws(P, ws, ws_bytes);
    if (!P->opts.differentiable) fail(MITNC_INVALID_ARG, "plan was not created with differentiable = 1");
    if (!w || !grad) fail(MITNC_INVALID_ARG, "null argument");
    uint64_t n_slices = 1ull << P->S;
    if (s0 >= s1 || s1 > n_slices) fail(MITNC_INVALID_ARG, "slice range out of bounds");
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    const int root = P->steps.back().out;
    uint64_t sl = s1;
    // Accumulators of the deferral roots start each run of slices at zero.
    auto clear_acc = [&](int node) {
      hip_check(hipMemsetAsync(base + P->off_adj + P->adj_offset[node], 0, 8ull << P->nodes[node].rank, s),
                "adjoint accumulator reset");
    };
    for (size_t g = 1; g < P->rev_groups.size(); ++g) clear_acc(P->rev_groups[g].root);
    std::function<void(int)> run_group = [&](int gi) {
      const mitnc_plan::RevGroup& G = P->rev_groups[gi];
      for (const mitnc_plan::RevLevel& L : G.levels) {
        for (int ri : L.big) {
          const RevOp& r = P->rev[ri];
          StepDesc d = r.d;
          char* adj_c = base + P->off_adj + P->adj_offset[P->steps[r.step].out];
          char* other = node_value_ptr(P, base, r.other, sl);
          d.A = r.adj_is_a ? adj_c : other;
          d.B = r.adj_is_a ? other : adj_c;
          d.C = base + P->off_adj +
                (P->defer_group[r.target] >= 0 ? P->adj_term_offset[r.target] : P->adj_offset[r.target]);
          d.acc = nullptr;
          d.part = (float*)(base + P->off_part);
          d.stats = nullptr;
          d.mode = EPI_STORE;
          d.prec = MITNC_C64;
          d.out_scale = 1.f;
          d.acc_scale = 1.0;
          hip_check(launch_step(r.kclass, d, s), "reverse kernel launch");
        }
        if (L.small_blocks)
          hip_check(launch_small_multi((const SmallRevOp*)(base + P->off_rtab), (const uint32_t*)(base + P->off_rblock),
                                       L.small_first, L.small_blocks, base, sl, s),
                    "reverse small-step launch");
      }
      for (int c : G.children) {  // this slice's term of each child's adjoint
        const int v = P->rev_groups[c].root;
        hip_check(launch_merge_add(MITNC_C64, base + P->off_adj + P->adj_offset[v],
                                   base + P->off_adj + P->adj_term_offset[v], 1ull << P->nodes[v].rank, nullptr, s),
                  "adjoint accumulation");
      }
      if (G.grad_count)
        hip_check(launch_grad((const GradEntry*)(base + P->off_gtab) + G.grad_first, (int)G.grad_count, base, sl,
                              grad, s),
                  "gradient accumulation");
      for (int c : G.children) {
        const mitnc_plan::RevGroup& C = P->rev_groups[c];
        if (sl == s0 || (sl & ((1ull << C.lo) - 1)) == 0) {
          run_group(c);
          clear_acc(C.root);
        }
      }
    };
    // Slices run from the last to the first: when the workspace still holds
    // the values of the last slice (the forward pass that produced the
    // amplitudes ended there), its recomputation is skipped.  Going from
    // slice s + 1 down to s changes the slice-id bits 0 .. ctz(s + 1), so a
    // node is recomputed when its lowest sliced bit is at most that.
    while (sl-- > s0) {
      // forward: recompute the nodes whose sliced indices changed (the root's
      // value itself is not needed)
      int level;
      if (sl == s1 - 1) level = P->valid_slice == (int64_t)sl ? -1 : kLevelFirst;
      else level = __builtin_ctzll(sl + 1);
      for (auto& st : P->steps) {
        if (st.root || P->nodes[st.out].lo > level) continue;
        launch_plan_step(P, st, base, sl, nullptr, s, MITNC_C64, false);
      }
      P->valid_slice = (int64_t)sl;
      // reverse: group 0 for every slice; a deferral root's group once its
      // run of slices is complete (the slice id a multiple of 2^lo, or the
      // range's first slice; slices go downwards)
      hip_check(launch_seed(w, (float*)(base + P->off_adj + P->adj_offset[root]), P->result_elems, s), "seed");
      run_group(0);
    }
  });
}

int32_t mitnc_plan_set_gates(mitnc_plan* P, void* ws, size_t ws_bytes, const double* mats, void* stream) {
  return guarded([&] {
    check_ws(P, ws, ws_bytes);
    if (!mats) fail(MITNC_INVALID_ARG, "null matrices");
    if (P->opts.precision != MITNC_C64) fail(MITNC_UNSUPPORTED, "gate updates need a complex64 plan");
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    int g = 0;
    for (int i = 0; i < P->n_leaves; ++i) {
      if (!P->leaf_is_1q[i]) continue;
      std::vector<float>& h = P->leaf_data[i];
      for (int e = 0; e < 4; ++e) {
        h[2 * e] = (float)mats[8 * g + 2 * e];
        h[2 * e + 1] = (float)mats[8 * g + 2 * e + 1];
      }
      hip_check(hipMemcpyAsync(base + P->nodes[i].offset, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice,
                               s),
                "gate upload");
      ++g;
    }
    P->valid_slice = -1;
    hip_check(hipStreamSynchronize(s), "gate upload sync");
  });
}

}  // extern "C"

// One pairwise contraction (mitnc_contract and its allocation-free form).
static void contract_impl(const void* A, int32_t ra, const int64_t* la, const void* B, int32_t rb,
                          const int64_t* lb, void* C, int32_t rc, const int64_t* lc, int32_t precision,
                          float out_scale, int32_t kernel, void* work, size_t work_bytes, size_t* work_bytes_needed,
                          void* stream) {
  if (ra < 0 || rb < 0 || rc < 0 || ra > 32 || rb > 32 || rc > 32) fail(MITNC_INVALID_ARG, "bad rank");
  if ((ra && !la) || (rb && !lb) || (rc && !lc)) fail(MITNC_INVALID_ARG, "null labels");
  if (precision != MITNC_C64 && precision != MITNC_CF16 && precision != MITNC_CBF16)
    fail(MITNC_INVALID_ARG, "unknown precision");
  // Reuse the plan step builder on a two-leaf pseudo-plan.
  mitnc_plan P;
  P.nodes.resize(3);
  auto setn = [](PlanNode& nd, int r, const int64_t* l) {
    for (int i = 0; i < r; ++i) {
      nd.labels.push_back(l[i]);
      nd.pos.push_back(i);
    }
    nd.rank = r;
  };
  setn(P.nodes[0], ra, la);
  setn(P.nodes[1], rb, lb);
  std::map<int64_t, int> cnt;
  for (int i = 0; i < ra; ++i) cnt[la[i]] |= 1;
  for (int i = 0; i < rb; ++i) cnt[lb[i]] |= 2;
  std::vector<int64_t> cl(lc, lc + rc);
  for (auto x : cl)
    if (!cnt.count(x)) fail(MITNC_INVALID_ARG, "output label not in any operand");
  for (size_t i = 0; i < cl.size(); ++i)
    for (size_t j = i + 1; j < cl.size(); ++j)
      if (cl[i] == cl[j]) fail(MITNC_INVALID_ARG, "duplicate output label");
  PlanStep st;
  st.a = 0;
  st.b = 1;
  st.out = 2;
  st.root = false;
  build_step_for(&P, st, cl, &cl, kernel, precision);
  if (work_bytes_needed) *work_bytes_needed = st.part_bytes;
  if (!A && !B && !C) return;  // size query
  if (!A || !B || !C) fail(MITNC_INVALID_ARG, "null tensor");
  if (st.part_bytes > 0 && (!work || work_bytes < st.part_bytes))
    fail(MITNC_WORKSPACE_TOO_SMALL, "split-K work buffer too small");
  StepDesc d = st.d;
  d.A = st.swapped ? B : A;
  d.B = st.swapped ? A : B;
  d.C = C;
  d.acc = nullptr;
  d.part = (float*)work;
  d.stats = nullptr;
  d.mode = EPI_STORE;
  d.prec = precision;
  d.out_scale = out_scale;
  d.acc_scale = 1.0;
  hip_check(launch_step(st.kclass, d, (hipStream_t)stream), "kernel launch");
}

// Device scratch of the allocation-free entry point: the split-K partial
// sums (one FP32 complex per split and output entry).  Each GPU the library
// runs on holds its own copy until the process ends.  Host code must not
// pass `scratch` itself to a kernel (on the host it is only a stand-in):
// the device address comes from hipGetSymbolAddress, once per device.
static constexpr size_t kScratchBytes = 32ull << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_dev[256];

static void* scratch_for_current_device() {
  int dev = -1;
  hip_check(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= 256) fail(MITNC_UNSUPPORTED, "device id out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch symbol address");
    if (!ptr) fail(MITNC_HIP_ERROR, "scratch symbol address is null");
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

extern "C" {

int32_t mitnc_contract(const void* A, int32_t ra, const int64_t* la, const void* B, int32_t rb, const int64_t* lb,
                       void* C, int32_t rc, const int64_t* lc, int32_t precision, float out_scale, int32_t kernel,
                       void* work, size_t work_bytes, size_t* work_bytes_needed, void* stream) {
  return guarded([&] {
    contract_impl(A, ra, la, B, rb, lb, C, rc, lc, precision, out_scale, kernel, work, work_bytes,
                  work_bytes_needed, stream);
  });
}

int32_t mitnc_contract_noalloc(const void* A, int32_t ra, const int64_t* la, const void* B, int32_t rb,
                               const int64_t* lb, void* C, int32_t rc, const int64_t* lc, int32_t precision,
                               float out_scale, int32_t kernel, void* stream) {
  return guarded([&] {
    if (!A || !B || !C) fail(MITNC_INVALID_ARG, "null tensor");
    size_t need = 0;
    contract_impl(nullptr, ra, la, nullptr, rb, lb, nullptr, rc, lc, precision, out_scale, kernel, nullptr, 0,
                  &need, stream);
    if (need > kScratchBytes)
      fail(MITNC_WORKSPACE_TOO_SMALL, "split-K partials need " + std::to_string(need) +
                                          " bytes, more than the fixed scratch of " + std::to_string(kScratchBytes) +
                                          " bytes; use mitnc_contract with a work buffer");
    void* work = need ? scratch_for_current_device() : nullptr;
    contract_impl(A, ra, la, B, rb, lb, C, rc, lc, precision, out_scale, kernel, work, kScratchBytes, nullptr,
                  stream);
  });
}

int32_t mitnc_plan_timing(mitnc_plan* P, int32_t enable) {
  return guarded([&] {
    if (!P) fail(MITNC_INVALID_ARG, "null plan");
    P->timing = enable != 0;
    P->ev_used = 0;
    P->ev_step.clear();
  });
}

int32_t mitnc_plan_timing_read(mitnc_plan* P, double* ms, double* launches, double* flops, double* bytes) {
  return guarded([&] {
    if (!P || !ms || !launches || !flops || !bytes) fail(MITNC_INVALID_ARG, "null argument");
    for (int c = 0; c < 8; ++c) ms[c] = launches[c] = flops[c] = bytes[c] = 0;
    for (size_t i = 0; i < P->ev_used; ++i) {
      hipEvent_t e0 = (hipEvent_t)P->ev_pool[2 * i], e1 = (hipEvent_t)P->ev_pool[2 * i + 1];
      hip_check(hipEventSynchronize(e1), "event sync");
      float t = 0;
      hip_check(hipEventElapsedTime(&t, e0, e1), "event time");
      const int id = P->ev_step[i];
      if (id > kMergeEvent && id <= kFwdEvent) {  // batched forward SMALL steps of one level
        const mitnc_plan::FwdBatch& b = P->fwd_runs[0].levels[kFwdEvent - id];
        ms[MITNC_K_SMALL] += t;
        launches[MITNC_K_SMALL] += 1;
        flops[MITNC_K_SMALL] += b.flops;
        bytes[MITNC_K_SMALL] += b.bytes;
        continue;
      }
      if (id <= kMergeEvent) {  // merge addition: acc += term, 2 real flops and 3 accesses per entry
        const int v = kMergeEvent - id;
        const double n = std::ldexp(1.0, P->nodes[P->steps[v / 4].out].full_rank);
        ms[kMergeClass] += t;
        launches[kMergeClass] += 1;
        flops[kMergeClass] += 2 * n;
        bytes[kMergeClass] += 3 * n * (v % 4 == MITNC_C64 ? 8 : 4);
        continue;
      }
      if (id < 0) {  // fused section: its own class
        const PlanSection& sec = P->sections[-1 - id];
        ms[kSectionClass] += t;
        launches[kSectionClass] += 1;
        flops[kSectionClass] += sec.flops;
        bytes[kSectionClass] += sec.bytes;
        continue;
      }
      const PlanStep& st = P->steps[id];
      ms[st.kclass] += t;
      launches[st.kclass] += 1;
      flops[st.kclass] += st.flops;
      bytes[st.kclass] += st.bytes;
    }
  });
}

void mitnc_plan_destroy(mitnc_plan* plan) { delete plan; }
void mitnc_network_destroy(mitnc_network* net) { delete net; }

}  // extern "C"
