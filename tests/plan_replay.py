"""Host re-execution of a plan's schedule, for CPU tests of the planner.

Test infrastructure only.  It reads a plan's address maps, node storage and
recompute levels through the library's introspection entry points and
replays the launch schedule on a complex128 copy of the workspace with
numpy: every step gathers its operands through the bit-position tables,
contracts them (einsum over batch, m, k, n) and scatters the result, the
last step of a slice adding into the result.  Independent of the kernels,
it checks the host logic that decides what the kernels are given: layouts,
workspace offsets (overlaps corrupt values), reuse levels, hoisting and the
per-slice sub-tensor offsets.
"""
import numpy as np


def _scatter(vals, pos):
    r = np.zeros(vals.shape, dtype=np.int64)
    for i, p in enumerate(pos):
        r |= ((vals >> i) & 1) << p
    return r


class PlanReplay:
    def __init__(self, plan):
        self.plan = plan
        st = plan.stats
        self.n_steps = st.n_steps
        self.steps = [plan.step_info(i) for i in range(self.n_steps)]
        n_nodes = self.steps[-1]["out"] + 1
        self.nodes = [plan.node_info(i) for i in range(n_nodes)]
        self.ws = np.zeros(int(st.workspace_bytes) // 8 + 1, dtype=np.complex128)
        self.n_leaves = sum(1 for nd in self.nodes if nd["is_leaf"])
        for i in range(self.n_leaves):
            z = plan.leaf_data(i)
            o = self.nodes[i]["ws_offset"] // 8
            self.ws[o:o + z.size] = z
        self.result_elems = int(st.result_elems)
        self.executed = 0  # step executions so far

    def _ptr(self, node, s, operand):
        nd = self.nodes[node]
        e = sum(((s >> b) & 1) << p for b, p in nd["slice_bits"]) if operand else 0
        return nd["ws_offset"] // 8 + e

    def _contract(self, st, a_flat, b_flat):
        """One step on flat operands (address bits as in the step's maps);
        returns (output address of each entry, value)."""
        b_, m_, k_, n_ = (np.arange(1 << st[x]) for x in ("bb", "mb", "kb", "nb"))
        ia = (_scatter(b_, st["ab"])[:, None, None] + _scatter(m_, st["am"])[None, :, None]
              + _scatter(k_, st["ak"])[None, None, :])
        ib = (_scatter(b_, st["bbt"])[:, None, None] + _scatter(k_, st["bk"])[None, :, None]
              + _scatter(n_, st["bn"])[None, None, :])
        ic = (_scatter(b_, st["cb"])[:, None, None] + _scatter(m_, st["cm"])[None, :, None]
              + _scatter(n_, st["cn"])[None, None, :])
        c = np.einsum("bmk,bkn->bmn", a_flat[ia], b_flat[ib])
        return ic.reshape(-1), c.reshape(-1)

    def _operand(self, node, s):
        nd = self.nodes[node]
        o = self._ptr(node, s, True)
        return self.ws[o:o + (1 << nd["full_rank"])]  # a view; only the slice's address bits are used

    def run(self, s0, s1):
        """Slices s0 .. s1-1 in order, as the library runs them (its launch
        list, mitnc_plan_schedule); returns the complex128 sum of their
        results.  A fused section runs where its last step is; its
        intermediates live outside the workspace, as on the GPU.  A merge
        term (mode 2) is written to the node's term buffer and then added
        into the node's accumulator."""
        acc = np.zeros(self.result_elems, dtype=np.complex128)
        sections = {}
        for i, st in enumerate(self.steps):
            if st["section"] >= 0:
                sections.setdefault(st["section"], []).append(i)
        for s, i, mode in self.plan.schedule(s0, s1):
            st = self.steps[i]
            if st["section"] >= 0 and st["section_pos"] != st["section_len"] - 1:
                continue  # runs with its section
            chain = sections[st["section"]] if st["section"] >= 0 else [i]
            a = self._operand(self.steps[chain[0]]["a"], s)
            for j in chain:
                sj = self.steps[j]
                self.executed += 1
                idx, val = self._contract(sj, a, self._operand(sj["b"], s))
                out = np.zeros(1 << self.nodes[sj["out"]]["full_rank"], dtype=np.complex128)
                out[idx] = val
                a = out
            if st["root"]:
                np.add.at(acc, idx, val)
            elif mode == 2:
                nd = self.nodes[st["out"]]
                size = 1 << nd["full_rank"]
                t = nd["merge_tmp_offset"] // 8
                o = self._ptr(st["out"], s, False)
                self.ws[t + idx] = val
                self.ws[o:o + size] += self.ws[t:t + size]
            else:
                o = self._ptr(st["out"], s, False)
                self.ws[o + idx] = val
        return acc
