"""Plain FP64 CPU oracle for sliced tensor-network contraction of random circuits.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never calls it, shares no code with it, and this package imports nothing from
the GPU library.  Its inputs come from the shared seeded generator package
``synth`` (which holds no contraction arithmetic).

What it computes (paper: Background, "Challenges of Large Tensor Networks";
Data Reuse Strategy, Sec. III-A):
  * a circuit becomes a tensor network whose edges are qubit wire segments; a
    pairwise contraction sums over the shared edges, done here as
    transpose + reshape + matmul (the TTGT form the paper describes);
  * slicing fixes the value of chosen edges; the 2^s sub-networks are
    contracted independently and summed (exact by distributivity);
  * brute-force state-vector amplitudes for small circuits;
  * the gradient of sum_b log|a_b|^2 with respect to every single-qubit gate
    tensor by reverse-mode contraction (not in the paper; problem definition of
    the differentiation form), plus the state-vector environment formula;
  * error metrics (relative L2, overlap fidelity, linear XEB ratio);
  * the lifetimes of sliced indices over a path (Sec. III-B), which fix how
    often the spindle (pre- plus post-lifetime reuse) needs each step.

Every function states the passage it follows.  Parity status of each part is
recorded in the module headers; all parts are pinned by ``tests/test_oracle_*``.
"""
from .network import Network, build_network, wire_label, BATCH  # noqa: F401
from .contract import (  # noqa: F401
    contract_pair, contract_network, contract_sliced, slice_leaves, amplitudes,
    count_contraction_flops,
)
from .planning import (  # noqa: F401
    greedy_path, random_greedy_path, path_stats, choose_slices, index_overhead, sliced_lifetimes,
)
from .statevector import sv_state, sv_amplitudes, sv_gate_gradients  # noqa: F401
from .grad import tn_gate_gradients, loss_log_abs2, torch_convention_grad  # noqa: F401
from .metrics import rel_l2, overlap_fidelity, xeb_ratio  # noqa: F401
