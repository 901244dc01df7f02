// Accumulation kernel of the post-lifetime merge (Sec. III-B): a merge
// accumulator (a node whose sliced index's lifetime has ended) receives its
// later terms through acc += term.  Elementwise and HBM bound: 3 x 8 bytes
// (complex64) or 3 x 4 bytes (FP16/BF16 storage) per entry; both tensors
// carry the node's one exponent, so FP16/BF16 terms add as stored.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace mitnc {

namespace {

__device__ __forceinline__ float h2f(uint32_t h) { return (float)__builtin_bit_cast(_Float16, (uint16_t)h); }
__device__ __forceinline__ uint32_t f2h(float f) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f); }
// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint32_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// One stored complex entry of 16-bit storage: (re, im) in the low / high half.
template <int P>
__device__ __forceinline__ uint32_t add_half(uint32_t a, uint32_t b, float& m) {
  float ar, ai, br, bi;
  if constexpr (P == MITNC_CF16) {
    ar = h2f(a & 0xffffu), ai = h2f(a >> 16), br = h2f(b & 0xffffu), bi = h2f(b >> 16);
  } else {
    ar = __uint_as_float(a << 16), ai = __uint_as_float(a & 0xffff0000u);
    br = __uint_as_float(b << 16), bi = __uint_as_float(b & 0xffff0000u);
  }
  const float re = ar + br, im = ai + bi;
  const uint32_t w = P == MITNC_CF16 ? (f2h(re) | (f2h(im) << 16)) : (f2bf(re) | (f2bf(im) << 16));
  // the magnitude recorded is the stored one (FP16 overflow shows as inf)
  float sr, si;
  if constexpr (P == MITNC_CF16) sr = h2f(w & 0xffffu), si = h2f(w >> 16);
  else sr = __uint_as_float(w << 16), si = __uint_as_float(w & 0xffff0000u);
  const float x = fmaxf(fabsf(sr), fabsf(si));
  m = (isfinite(sr) && isfinite(si)) ? fmaxf(m, x) : __builtin_inff();
  return w;
}

__device__ __forceinline__ float mag(float a, float b, float m) {
  return (isfinite(a) && isfinite(b)) ? fmaxf(m, fmaxf(fabsf(a), fabsf(b))) : __builtin_inff();
}

// 16 bytes per lane and iteration (2 complex64 or 4 16-bit entries); n16:
// number of 16-byte groups.  The largest stored |Re|, |Im| is raised into
// *slot (float bits; at most one atomic per workgroup).
template <int P>
__global__ __launch_bounds__(256) void k_merge_add(uint4* acc, const uint4* term, uint64_t n16, unsigned int* slot) {
  float m = 0.f;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    uint4 a = acc[i];
    const uint4 b = term[i];
    if constexpr (P == MITNC_C64) {
      float4 x = __builtin_bit_cast(float4, a);
      const float4 y = __builtin_bit_cast(float4, b);
      x.x += y.x;
      x.y += y.y;
      x.z += y.z;
      x.w += y.w;
      m = mag(x.x, x.y, m);
      m = mag(x.z, x.w, m);
      a = __builtin_bit_cast(uint4, x);
    } else {
      a.x = add_half<P>(a.x, b.x, m);
      a.y = add_half<P>(a.y, b.y, m);
      a.z = add_half<P>(a.z, b.z, m);
      a.w = add_half<P>(a.w, b.w, m);
    }
    acc[i] = a;
  }
  if (!slot) return;
  __shared__ float red[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    const unsigned int v = __float_as_uint(m);
    if (m > 0.f && __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) atomicMax(slot, v);
  }
}

// Tensors of fewer than one 16-byte group: one thread per entry.
template <int P>
__global__ __launch_bounds__(64) void k_merge_add_small(void* acc, const void* term, uint64_t n, unsigned int* slot) {
  const uint64_t i = threadIdx.x;
  float m = 0.f;
  if (i < n) {
    if constexpr (P == MITNC_C64) {
      float2 a = reinterpret_cast<float2*>(acc)[i];
      const float2 b = reinterpret_cast<const float2*>(term)[i];
      a.x += b.x;
      a.y += b.y;
      m = mag(a.x, a.y, m);
      reinterpret_cast<float2*>(acc)[i] = a;
    } else {
      uint32_t* pa = reinterpret_cast<uint32_t*>(acc);
      pa[i] = add_half<P>(pa[i], reinterpret_cast<const uint32_t*>(term)[i], m);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (threadIdx.x == 0 && slot && m > 0.f) atomicMax(slot, __float_as_uint(m));
}

template <int P>
hipError_t launch_merge_add_p(void* acc, const void* term, uint64_t n, unsigned int* slot, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1) {
  const uint64_t per16 = P == MITNC_C64 ? 2 : 4;  // complex entries per 16 bytes
  if (n < per16) {
    if (n == 0 || n > 64) return hipErrorInvalidValue;
    hipExtLaunchKernelGGL(k_merge_add_small<P>, dim3(1), dim3(64), 0, s, ev0, ev1, 0, acc, term, n, slot);
    return hipGetLastError();
  }
  if (n % per16 || (reinterpret_cast<uintptr_t>(acc) | reinterpret_cast<uintptr_t>(term)) % 16)
    return hipErrorInvalidValue;
  const uint64_t n16 = n / per16;
  // About 8 groups per thread, at most 2^15 workgroups (grid-stride beyond).
  const uint64_t blocks = std::min<uint64_t>(32768, std::max<uint64_t>(1, (n16 + 2047) / 2048));
  hipExtLaunchKernelGGL(k_merge_add<P>, dim3((unsigned)blocks), dim3(256), 0, s, ev0, ev1, 0,
                        reinterpret_cast<uint4*>(acc), reinterpret_cast<const uint4*>(term), n16, slot);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_merge_add(int prec, void* acc, const void* term, uint64_t n, unsigned int* stats_slot,
                            hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  switch (prec) {
    case MITNC_C64: return launch_merge_add_p<MITNC_C64>(acc, term, n, stats_slot, s, ev0, ev1);
    case MITNC_CF16: return launch_merge_add_p<MITNC_CF16>(acc, term, n, stats_slot, s, ev0, ev1);
    case MITNC_CBF16: return launch_merge_add_p<MITNC_CBF16>(acc, term, n, stats_slot, s, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mitnc
