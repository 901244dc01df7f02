// Kernel launch interface (host side of kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/mitnc.h"
#include "step.hpp"

namespace mitnc {

// Launches the kernel(s) of one contraction step of class `kclass` on stream
// `s` (for split-K: the partial-tile kernel, then the FP64 reduction).
// With ev0/ev1 given, the main kernel (not a split-K reduction) is launched
// with hipExtLaunchKernelGGL so that the pair brackets its execution.
hipError_t launch_step(int kclass, const StepDesc& d, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);

// Launches a fused stem section (checks the tile geometry it assumes).
hipError_t launch_section(const SectionDesc& sd, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Reverse pass helpers: adj = complex64(w) for n entries; gradient
// accumulation of the single-qubit gate leaf adjoints of slice `slice`.
hipError_t launch_seed(const double* w, float* adj, uint64_t n, hipStream_t s);
// Batched SMALL reverse ops: workgroups [first, first + blocks) of the block
// table block_op (entries index ops), operands relative to the workspace ws.
hipError_t launch_small_multi(const SmallRevOp* ops, const uint32_t* block_op, uint32_t first, uint32_t blocks,
                              char* ws, uint64_t slice, hipStream_t s);
// Batched forward SMALL steps (any precision): workgroups [first, first +
// blocks) of the block table; stats: the per-step maxima (may be null).
hipError_t launch_small_fwd(int prec, const SmallFwdOp* ops, const uint32_t* block_op, uint32_t first, uint32_t blocks,
                            char* ws, float* stats, uint64_t slice, hipStream_t s);
// acc += src over n complex128 entries (device pointers).
hipError_t launch_accumulate(double* acc, const double* src, uint64_t n, hipStream_t s);
// Post-lifetime merge: acc += term over n complex entries stored in
// precision prec (16-byte aligned device pointers for n >= 2 / 4 entries);
// raises *stats_slot (may be null) to the largest stored |Re|, |Im|.
hipError_t launch_merge_add(int prec, void* acc, const void* term, uint64_t n, unsigned int* stats_slot,
                            hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_grad(const GradEntry* tab, int n_entries, const char* ws, uint64_t slice, double* grad,
                       hipStream_t s);

}  // namespace mitnc
