// Contraction kernels for gfx950 (CDNA4).
//
// Every kernel computes one pairwise contraction described by a StepDesc:
//   C[b, m, n] = sum_k A[b, m, k] * B[b, k, n]     (complex)
// with each logical bit scattered to an arbitrary address bit of each operand
// (TTGT of Sec. II-A with the transposes fused into the loads, Sec. V-A).
//
// Storage precision P: 0 = complex64 (interleaved float), 1 = complex FP16,
// 2 = complex BF16 (interleaved 16-bit halves, one 32-bit word per entry).
// Arithmetic accumulates in FP32.  A stored FP16/BF16 tensor is a mantissa
// tensor with a per-tensor power-of-two exponent kept by the host plan: the
// epilogue multiplies by out_scale (2^(eA + eB - eC)) before rounding, and the
// last step of a slice adds result * acc_scale (2^(eA + eB)) into the FP64
// result.
//
// The bit-position tables of the descriptor are copied to LDS once per
// workgroup; every address decode then reads LDS (a dynamically indexed
// kernel argument would cost a global load per bit).
//
// Flop counts reported by the library use the 4M convention, 8 M K N real
// flops per complex contraction, whichever split executes.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <type_traits>

#include "kernels.hpp"

namespace mitnc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

static_assert(offsetof(StepDesc, am) % 4 == 0, "tables must be dword aligned");
static_assert(offsetof(StepDesc, hk) + 8 - offsetof(StepDesc, am) == TAB_BYTES, "table layout");
static_assert(offsetof(StepDesc, ha_row) - offsetof(StepDesc, am) == T_HAROW &&
                  offsetof(StepDesc, hb_row) - offsetof(StepDesc, am) == T_HBROW &&
                  offsetof(StepDesc, hk) - offsetof(StepDesc, am) == T_HK,
              "table offsets");

__device__ __forceinline__ void load_tables(const StepDesc& d, uint8_t* tab) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(d.am);
  uint32_t* dst = reinterpret_cast<uint32_t*>(tab);
  for (int i = threadIdx.x; i < TAB_BYTES / 4; i += blockDim.x) dst[i] = src[i];
}

// Deposits the low n bits of x at the address bits pos[0..n) (n <= 32).
__device__ __forceinline__ uint64_t scatter_bits(uint64_t x, const uint8_t* pos, int n) {
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i)
    if (i < n) r |= ((x >> i) & 1ull) << pos[i];
  return r;
}

// scatter_bits for n <= MAXN with no branches: every position byte is read
// (index clamped to stay inside pos[0..n)), so the LDS reads issue back to
// back and are waited for once (a per-bit branch on i < n serialises them).
template <int MAXN>
__device__ __forceinline__ uint64_t scatter_bits_n(uint64_t x, const uint8_t* pos, int n) {
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < MAXN; ++i) {
    const bool on = i < n;
    const uint32_t p = pos[on ? i : 0];
    r |= (on ? ((x >> i) & 1ull) : 0ull) << p;
  }
  return r;
}

// scatter_bits of a wave-uniform x, computed across the lanes: lane i
// deposits bit i, an OR-reduction over the wave combines them (one LDS read
// per lane instead of n dependent ones).  Every lane of the wave must call it
// with the same arguments; every lane gets the result.  n <= 32.
__device__ __forceinline__ uint64_t wave_scatter(uint64_t x, const uint8_t* pos, int n) {
  const int l = threadIdx.x & 63;
  const bool on = l < n;
  const uint32_t p = pos[on ? l : 0];
  uint64_t t = on ? (((x >> l) & 1ull) << p) : 0ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)t, o), hi = __shfl_xor((uint32_t)(t >> 32), o);
    t |= ((uint64_t)hi << 32) | lo;
  }
  return t;
}

// gather_bits for n <= MAXN with no branches (as scatter_bits_n).
template <int MAXN>
__device__ __forceinline__ uint64_t gather_bits_n(uint64_t a, const uint8_t* pos, int n) {
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < MAXN; ++i) {
    const bool on = i < n;
    const uint32_t p = pos[on ? i : 0];
    r |= (on ? ((a >> p) & 1ull) : 0ull) << i;
  }
  return r;
}

// Extracts the address bits pos[0..n) of a into the low n bits (n <= 32).
__device__ __forceinline__ uint64_t gather_bits(uint64_t a, const uint8_t* pos, int n) {
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i)
    if (i < n) r |= ((a >> pos[i]) & 1ull) << i;
  return r;
}

// A wave-uniform 64-bit value moved to scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
}

// ---------------------------------------------------------------- element I/O
__device__ __forceinline__ float h_to_f(uint32_t bits16) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}
__device__ __forceinline__ uint32_t f_to_h(float f) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f);
}
// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint32_t f_to_bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

template <int P>
__device__ __forceinline__ float2 unpack(uint32_t w) {
  if constexpr (P == 1) return make_float2(h_to_f(w & 0xffffu), h_to_f(w >> 16));
  else return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}

template <int P>
__device__ __forceinline__ uint32_t pack(float2 v) {
  if constexpr (P == 1) return f_to_h(v.x) | (f_to_h(v.y) << 16);
  else return f_to_bf(v.x) | (f_to_bf(v.y) << 16);
}

template <int P>
__device__ __forceinline__ float2 load_c(const void* p, uint64_t i) {
  if constexpr (P == 0) return reinterpret_cast<const float2*>(p)[i];
  else return unpack<P>(reinterpret_cast<const uint32_t*>(p)[i]);
}

__device__ __forceinline__ float absmax2(float2 v) {
  float a = fmaxf(fabsf(v.x), fabsf(v.y));
  return (isfinite(v.x) && isfinite(v.y)) ? a : __builtin_inff();
}

// Writes one output entry; returns the magnitude stored (for statistics).
template <int P>
__device__ __forceinline__ float epilogue_store(const StepDesc& d, uint64_t addr, float2 v, uint64_t split,
                                                uint64_t c_elems) {
  if (d.mode == EPI_STORE) {
    if constexpr (P == 0) {
      reinterpret_cast<float2*>(d.C)[addr] = v;
      return absmax2(v);
    } else {
      const float2 s = make_float2(v.x * d.out_scale, v.y * d.out_scale);
      reinterpret_cast<uint32_t*>(d.C)[addr] = pack<P>(s);
      return absmax2(s);
    }
  } else if (d.mode == EPI_ACC64) {
    double2* acc = reinterpret_cast<double2*>(d.acc);
    double2 o = acc[addr];
    o.x += (double)v.x * d.acc_scale;
    o.y += (double)v.y * d.acc_scale;
    acc[addr] = o;
    return 0.f;  // nothing stored in 16 bits
  } else {
    reinterpret_cast<float2*>(d.part)[split * c_elems + addr] = v;
    return 0.f;
  }
}

// Raises the recorded maximum *slot to m (the bit pattern of a non-negative
// float orders like the float).  The recorded value only grows, so a plain
// read that already shows m or more makes the atomic unnecessary: with
// thousands of workgroups per launch, most skip it instead of queueing on
// one address.
__device__ __forceinline__ void raise_max(unsigned int* slot, float m) {
  const unsigned int v = __float_as_uint(m);
  if (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) atomicMax(slot, v);
}

// Per-step maximum of stored magnitudes: wave and workgroup reduction, at
// most one atomic per workgroup.  Every thread of the workgroup must call it.
__device__ __forceinline__ void record_max(const StepDesc& d, float m) {
  if (!d.stats) return;
  __shared__ float red[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    if (m > 0.f) raise_max(reinterpret_cast<unsigned int*>(d.stats) + d.step_index, m);
  }
}

// ---------------------------------------------------------------- small steps
// One thread per output entry, direct loads; correct for any shape.  Output
// entry c of C (address bits by the tables in LDS) from operands A, B.
// BOUNDED: small_bounded holds (the SMALL class limits), so the address
// helpers run with compile-time bounds and no branches.

template <bool BOUNDED>
__device__ __forceinline__ uint64_t sc_s(uint64_t x, const uint8_t* pos, int n) {
  if constexpr (BOUNDED) return scatter_bits_n<kSmallBits>(x, pos, n);
  else return scatter_bits(x, pos, n);
}
template <bool BOUNDED>
__device__ __forceinline__ uint64_t ga_s(uint64_t a, const uint8_t* pos, int n) {
  if constexpr (BOUNDED) return gather_bits_n<kSmallBits>(a, pos, n);
  else return gather_bits(a, pos, n);
}

template <int P, bool BOUNDED = false>
__device__ __forceinline__ float2 small_entry(const void* A, const void* B, const uint8_t* tab, int mb, int nb,
                                              int kb, int bb, uint64_t c) {
  const uint64_t m = ga_s<BOUNDED>(c, tab + T_CM, mb), n = ga_s<BOUNDED>(c, tab + T_CN, nb),
                 b = ga_s<BOUNDED>(c, tab + T_CB, bb);
  const uint64_t ao = sc_s<BOUNDED>(m, tab + T_AM, mb) + sc_s<BOUNDED>(b, tab + T_AB, bb);
  const uint64_t bo = sc_s<BOUNDED>(n, tab + T_BN, nb) + sc_s<BOUNDED>(b, tab + T_BB, bb);
  // The k loop runs in groups of up to 8 independent loads so that memory
  // latency is paid once per group rather than once per term.
  const int kl = kb < 3 ? kb : 3;
  const int KL = 1 << kl;
  uint32_t ak_lo[8], bk_lo[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if constexpr (BOUNDED) {
      ak_lo[j] = (uint32_t)scatter_bits_n<3>(j, tab + T_AK, kl);
      bk_lo[j] = (uint32_t)scatter_bits_n<3>(j, tab + T_BK, kl);
    } else {
      ak_lo[j] = (uint32_t)scatter_bits(j, tab + T_AK, kl);
      bk_lo[j] = (uint32_t)scatter_bits(j, tab + T_BK, kl);
    }
  }
  const uint64_t KH = 1ull << (kb - kl);
  float2 s = make_float2(0.f, 0.f);
  for (uint64_t kh = 0; kh < KH; ++kh) {
    uint64_t ah, bh;
    if constexpr (BOUNDED) {  // kb <= 6: at most 3 high k bits
      ah = ao + scatter_bits_n<3>(kh, tab + T_AK + kl, kb - kl);
      bh = bo + scatter_bits_n<3>(kh, tab + T_BK + kl, kb - kl);
    } else {
      ah = ao + scatter_bits(kh, tab + T_AK + kl, kb - kl);
      bh = bo + scatter_bits(kh, tab + T_BK + kl, kb - kl);
    }
    float2 a[8], bv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < KL) {
        a[j] = load_c<P>(A, ah + ak_lo[j]);
        bv[j] = load_c<P>(B, bh + bk_lo[j]);
      }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < KL) {
        s.x += a[j].x * bv[j].x - a[j].y * bv[j].y;
        s.y += a[j].x * bv[j].y + a[j].y * bv[j].x;
      }
  }
  return s;
}

template <int P, bool BOUNDED>
__global__ __launch_bounds__(256) void k_small(StepDesc d) {
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  load_tables(d, tab);
  __syncthreads();
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  const uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  float mx = 0.f;
  if (c < c_elems)
    mx = epilogue_store<P>(d, c, small_entry<P, BOUNDED>(d.A, d.B, tab, d.mb, d.nb, d.kb, d.bb, c), 0, c_elems);
  record_max(d, mx);
}

// Many independent SMALL steps of the reverse pass (complex64) in one
// launch: workgroup first + blockIdx.x of the block table names its op; the
// op's operands are workspace offsets, a sliced leaf operand is offset by
// the slice's values of its sliced indices.
__global__ __launch_bounds__(256) void k_small_multi(const SmallRevOp* ops, const uint32_t* block_op, uint32_t first,
                                                     char* ws, uint64_t slice) {
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  const uint32_t gb = first + blockIdx.x;
  const SmallRevOp& op = ops[block_op[gb]];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(op.d.am);
    uint32_t* dst = reinterpret_cast<uint32_t*>(tab);
    for (int i = threadIdx.x; i < TAB_BYTES / 4; i += blockDim.x) dst[i] = src[i];
  }
  const int mb = op.d.mb, nb = op.d.nb, kb = op.d.kb, bb = op.d.bb;
  uint64_t sl_off = 0;
  for (int j = 0; j < op.sl_n; ++j) sl_off |= ((slice >> op.sl_bit[j]) & 1ull) << op.sl_pos[j];
  const char* A = ws + op.a_off + (op.sl_which == 1 ? sl_off * 8 : 0);
  const char* B = ws + op.b_off + (op.sl_which == 2 ? sl_off * 8 : 0);
  float2* C = reinterpret_cast<float2*>(ws + op.c_off);
  __syncthreads();
  const uint64_t c_elems = 1ull << (mb + nb + bb);
  const uint64_t c = (uint64_t)(gb - op.block0) * 256 + threadIdx.x;
  if (c < c_elems) C[c] = small_entry<0, true>(A, B, tab, mb, nb, kb, bb, c);
}

// Many independent SMALL steps of the forward pass in one launch (the steps
// a slice range computes once, grouped by dependency level): workgroup first
// + blockIdx.x of the block table names its step; operands and output are
// workspace offsets, a sliced operand read at the slice's values of its
// sliced indices; the output goes through the step's epilogue (16-bit
// storage scaled by its out_scale) and its stored maximum into stats.
template <int P>
__global__ __launch_bounds__(256) void k_small_fwd(const SmallFwdOp* ops, const uint32_t* block_op, uint32_t first,
                                                   char* ws, float* stats, uint64_t slice) {
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  const uint32_t gb = first + blockIdx.x;
  const SmallFwdOp& op = ops[block_op[gb]];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(op.d.am);
    uint32_t* dst = reinterpret_cast<uint32_t*>(tab);
    for (int i = threadIdx.x; i < TAB_BYTES / 4; i += blockDim.x) dst[i] = src[i];
  }
  StepDesc d = op.d;
  d.C = ws + op.c_off;
  d.stats = stats;
  constexpr uint64_t ES = P == 0 ? 8 : 4;
  uint64_t sa = 0, sb = 0;
  for (int j = 0; j < op.na; ++j) sa |= ((slice >> op.a_bit[j]) & 1ull) << op.a_pos[j];
  for (int j = 0; j < op.nb; ++j) sb |= ((slice >> op.b_bit[j]) & 1ull) << op.b_pos[j];
  const void* A = ws + op.a_off + sa * ES;
  const void* B = ws + op.b_off + sb * ES;
  __syncthreads();
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  const uint64_t c = (uint64_t)(gb - op.block0) * 256 + threadIdx.x;
  float mx = 0.f;
  if (c < c_elems) mx = epilogue_store<P>(d, c, small_entry<P, true>(A, B, tab, d.mb, d.nb, d.kb, d.bb, c), 0, c_elems);
  record_max(d, mx);
}

hipError_t launch_small_fwd(int prec, const SmallFwdOp* ops, const uint32_t* block_op, uint32_t first, uint32_t blocks,
                            char* ws, float* stats, uint64_t slice, hipStream_t s) {
  if (!blocks) return hipSuccess;
  switch (prec) {
    case MITNC_C64:
      hipLaunchKernelGGL(k_small_fwd<0>, dim3(blocks), dim3(256), 0, s, ops, block_op, first, ws, stats, slice);
      break;
    case MITNC_CF16:
      hipLaunchKernelGGL(k_small_fwd<1>, dim3(blocks), dim3(256), 0, s, ops, block_op, first, ws, stats, slice);
      break;
    case MITNC_CBF16:
      hipLaunchKernelGGL(k_small_fwd<2>, dim3(blocks), dim3(256), 0, s, ops, block_op, first, ws, stats, slice);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Every op of the table satisfies small_bounded (the planner puts the others
// on single launches).
hipError_t launch_small_multi(const SmallRevOp* ops, const uint32_t* block_op, uint32_t first, uint32_t blocks,
                              char* ws, uint64_t slice, hipStream_t s) {
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(k_small_multi, dim3(blocks), dim3(256), 0, s, ops, block_op, first, ws, slice);
  return hipGetLastError();
}

// ---------------------------------------------------------------- skinny split-K
// C[b][m][n] = sum_k A[b][m][k] B[b][k][n] for M N <= 16 and long K (the
// adjoints of small tensors under a large one in the reverse pass).  A tile
// kernel would stage a mostly empty 16 x 16 tile per k step; here one wave
// per (k split, batch index) streams both operands from HBM with no LDS:
// lane = the six lowest k bits, kSkinnyUnroll values of the higher k bits
// per iteration ((M + N) * 4 independent loads per lane in flight), the whole
// M x N block of complex sums in registers, a shuffle reduction over the
// wave at the end.  Split partials go through the FP64 reduction of the
// split-K path.
// Address change of one step of a counter whose bits 2.. sit at positions
// pos[2..]: step setting bit j (and clearing bits 2..j-1), modulo 2^64.
__device__ __forceinline__ unsigned long long skinny_step_delta(const uint8_t* pos, int j) {
  unsigned long long v = 1ull << pos[j];
#pragma unroll
  for (int i = 2; i < 26; ++i) {  // branch-free: j <= 25 (k <= 32)
    const bool on = i < j;
    v -= on ? 1ull << pos[on ? i : 0] : 0ull;
  }
  return v;
}

template <int MB, int NB>
__global__ __launch_bounds__(64) void k_skinny(StepDesc d) {
  constexpr int M = 1 << MB, N = 1 << NB, U = kSkinnyUnroll, LB = kSkinnyLaneBits;
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  load_tables(d, tab);
  __syncthreads();
  const int lane = threadIdx.x;
  const int KH = d.kb - LB;        // high k bits
  const int hl = KH - d.ks_bits;   // log2 of high k values per split (>= 2)
  const uint64_t split = blockIdx.x, b = blockIdx.y;
  const float2* A = reinterpret_cast<const float2*>(d.A) + wave_scatter(b, tab + T_AB, d.bb) +
                    scatter_bits_n<LB>(lane, tab + T_AK, LB);
  const float2* B = reinterpret_cast<const float2*>(d.B) + wave_scatter(b, tab + T_BB, d.bb) +
                    scatter_bits_n<LB>(lane, tab + T_BK, LB);
  // Offsets, one scatter per entry into LDS (wave-uniform values computed
  // in scalar registers would spill them): every m in A and n in B, the four
  // values of the two lowest high-k bits (one iteration) in A and B, this
  // split's first high-k offsets (its run starts at split << hl), and the
  // address change of a counter step: going from h to h + 1 sets bit
  // j = ctz(h + 1) and clears the bits below it, i.e. adds 2^p(j) minus the
  // sum of 2^p(i), 2 <= i < j, whatever order the positions p are in (A and
  // B place the k bits differently, so a walk in address order would pair
  // different k values).
  enum { E_AM = 0, E_BN = 16, E_OA = 32, E_OB = 36, E_XA = 40, E_XB = 41, E_DA = 64, E_DB = 96, E_N = 128 };
  __shared__ unsigned long long offs[E_N];
  // Pass 1 (entries 0-63): one bounded scatter per lane, its operands
  // selected per entry; pass 2 (64-127): the counter-step deltas.  One job
  // shape per pass, no divergent branches around the LDS reads.
  {
    uint64_t x = 0;
    int off = T_AM, n = 0;
    const int e = lane;
    if (e < E_AM + M) {
      x = e - E_AM; off = T_AM; n = MB;
    } else if (e >= E_BN && e < E_BN + N) {
      x = e - E_BN; off = T_BN; n = NB;
    } else if (e >= E_OA && e < E_OA + 4) {
      x = e - E_OA; off = T_AK + LB; n = 2;
    } else if (e >= E_OB && e < E_OB + 4) {
      x = e - E_OB; off = T_BK + LB; n = 2;
    } else if (e == E_XA || e == E_XB) {
      x = split << hl; off = (e == E_XA ? T_AK : T_BK) + LB; n = KH;
    }
    offs[e] = scatter_bits_n<26>(x, tab + off, n);  // KH <= 26 (k <= 32)
    const int j = lane & 31;
    offs[E_DA + lane] = j < KH ? skinny_step_delta(tab + (lane < 32 ? T_AK : T_BK) + LB, j) : 0ull;
  }
  __syncthreads();
  uint64_t a_m[M], b_n[N], oa[U], ob[U];
#pragma unroll
  for (int m = 0; m < M; ++m) a_m[m] = offs[E_AM + m];
#pragma unroll
  for (int n = 0; n < N; ++n) b_n[n] = offs[E_BN + n];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    oa[u] = offs[E_OA + u];
    ob[u] = offs[E_OB + u];
  }
  uint64_t xa = offs[E_XA], xb = offs[E_XB];
  float2 acc[M][N];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int n = 0; n < N; ++n) acc[m][n] = make_float2(0.f, 0.f);
  const uint32_t iters = 1u << (hl - 2);
  for (uint32_t it = 0; it < iters; ++it) {
    float2 ra[U][M], rb[U][N];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int m = 0; m < M; ++m) ra[u][m] = A[xa + oa[u] + a_m[m]];
#pragma unroll
      for (int n = 0; n < N; ++n) rb[u][n] = B[xb + ob[u] + b_n[n]];
    }
    if (it + 1 < iters) {
      const int j = 2 + __builtin_ctz(it + 1);  // high-k bit the next iteration sets
      xa += offs[E_DA + j];
      xb += offs[E_DB + j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int n = 0; n < N; ++n) {
          acc[m][n].x += ra[u][m].x * rb[u][n].x - ra[u][m].y * rb[u][n].y;
          acc[m][n].y += ra[u][m].x * rb[u][n].y + ra[u][m].y * rb[u][n].x;
        }
  }
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        acc[m][n].x += __shfl_xor(acc[m][n].x, o);
        acc[m][n].y += __shfl_xor(acc[m][n].y, o);
      }
  // Every lane holds every sum; lane m N + n stores entry (m, n).
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  const uint64_t cb = wave_scatter(b, tab + T_CB, d.bb);
  float mx = 0.f;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int n = 0; n < N; ++n)
      if (lane == m * N + n) {
        const uint64_t c = cb + scatter_bits_n<MB>(m, tab + T_CM, MB) + scatter_bits_n<NB>(n, tab + T_CN, NB);
        mx = epilogue_store<0>(d, c, acc[m][n], split, c_elems);
      }
  if (d.stats) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0 && mx > 0.f)
      raise_max(reinterpret_cast<unsigned int*>(d.stats) + d.step_index, mx);
  }
}


// ---------------------------------------------------------------- stem steps
// A big tensor absorbs a small matrix (K <= 16, N <= 4): one thread per row m
// (and batch index), the small matrix in LDS.  Consecutive threads take
// consecutive m, whose bits are A's lowest non-contracted address bits, so
// loads and stores are coalesced whatever the bit positions of k and n.
template <int P, int KB, int NB>
__global__ __launch_bounds__(256) void k_stem(StepDesc d) {
  constexpr int K = 1 << KB, N = 1 << NB;
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  __shared__ float2 Bs[K * N];
  __shared__ uint32_t ka[K], nc[N];
  load_tables(d, tab);
  __syncthreads();
  const uint64_t batch = blockIdx.y;
  const int t = threadIdx.x;
  // Batch offsets across the wave (uniform, every lane here), the rest with
  // bounded branch-free scatters.
  const uint64_t ab = wave_scatter(batch, tab + T_AB, d.bb), bbo = wave_scatter(batch, tab + T_BB, d.bb),
                 cbo = wave_scatter(batch, tab + T_CB, d.bb);
  if (t < K * N) {
    const int k = t / N, n = t % N;
    Bs[t] = load_c<P>(d.B, bbo + scatter_bits_n<KB>(k, tab + T_BK, KB) + scatter_bits_n<NB>(n, tab + T_BN, NB));
  }
  if (t < K) ka[t] = (uint32_t)scatter_bits_n<KB>(t, tab + T_AK, KB);
  if (t < N) nc[t] = (uint32_t)scatter_bits_n<NB>(t, tab + T_CN, NB);
  __syncthreads();
  const int lowb = d.mb < 8 ? d.mb : 8;
  const uint64_t n_mhi = 1ull << (d.mb - lowb);
  const uint64_t a_lo = scatter_bits_n<8>(t, tab + T_AM, lowb), c_lo = scatter_bits_n<8>(t, tab + T_CM, lowb);
  float mx = 0.f;
  for (uint64_t mhi = blockIdx.x; t < (1 << lowb) && mhi < n_mhi; mhi += gridDim.x) {  // high m bits (uniform)
    // at most 24 high m bits (m <= 32)
    const uint64_t aoff = scatter_bits_n<24>(mhi, tab + T_AM + lowb, d.mb - lowb) + ab + a_lo;
    const uint64_t coff = scatter_bits_n<24>(mhi, tab + T_CM + lowb, d.mb - lowb) + cbo + c_lo;
    float2 a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = load_c<P>(d.A, aoff + ka[k]);
    const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
#pragma unroll
    for (int n = 0; n < N; ++n) {
      float2 s = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float2 b = Bs[k * N + n];
        s.x += a[k].x * b.x - a[k].y * b.y;
        s.y += a[k].x * b.y + a[k].y * b.x;
      }
      mx = fmaxf(mx, epilogue_store<P>(d, coff + nc[n], s, 0, c_elems));
    }
  }
  record_max(d, mx);
}

// ---------------------------------------------------------------- stream steps
// A large tensor absorbs a small matrix (K, N <= 64, K N <= 16 x 4 x 16): the
// HBM-bound steps that dominate a stem (Sec. V-A).  No LDS staging: the small
// matrix sits in registers for the whole kernel and every wave streams 16-row
// blocks of A from HBM straight into MFMA operands and writes C straight
// back.  The MFMA computes C^T = B^T A^T, so that the 16 lanes of a lane
// group walk 16 rows m of both A and C: the four lowest-address m bits.  The
// four lane groups take the two lowest-address k bits (loads) and n bits
// (stores), so with those six bits low in the address an instruction moves
// whole 128-byte lines.  3M split as in the tile kernels; padded k and n
// carry zero B entries and padded n are never stored.
//
// Each wave takes iters iterations of R row blocks (all R * KS loads of an
// iteration issued before the MFMAs; 8 loads of 8 bytes or 16 of 4 bytes per
// lane); the blocks of successive iterations are a window of all waves
// apart (see StreamLut).  Counters over scattered address bits advance by
// ((x | ~mask) + 1) & mask, in A (m bits are sorted by A position) and in C
// (the launcher requires its row bits in address order too).
// log2 of the row blocks times k steps one iteration loads (R * KS, or
// R * KS8 with 16-bit storage, when one row block has fewer k steps): the
// bytes a wave keeps in flight per iteration.
inline constexpr int kStreamRowsF = 3;
inline constexpr int kStreamRowsH = 3;
inline constexpr int ilog2c(int x) { return x > 1 ? 1 + ilog2c(x >> 1) : 0; }
static_assert(kStreamRowsF <= kStreamMinM - 4 && kStreamRowsH <= kStreamMinM - 4,
              "one iteration must not hold more row blocks than the smallest stream step has");
template <int P>
inline constexpr int stream_loads() { return 1 << kStreamRowsF; }

// Output entry of a stream step.  EPI: 0 = store, 1 = store and return the
// stored magnitude (statistics), 2 = add into the FP64 result.  out is the
// row block's base in C (EPI 0, 1) or in the result (EPI 2), off the lane's
// byte offset from it (32 bits: a scalar base plus a vector offset).
template <int P, int EPI>
inline constexpr uint32_t stream_out_bytes() { return EPI == 2 ? 16u : (P == 0 ? 8u : 4u); }

template <int P, int EPI>
__device__ __forceinline__ float stream_store(char* out, const StepDesc& d, uint32_t off, float2 v) {
  if constexpr (EPI == 2) {
    double2* acc = reinterpret_cast<double2*>(out + off);
    double2 o = *acc;
    o.x += (double)v.x * d.acc_scale;
    o.y += (double)v.y * d.acc_scale;
    *acc = o;
    return 0.f;
  } else {
    if constexpr (P == 0) {
      *reinterpret_cast<float2*>(out + off) = v;
    } else {
      v = make_float2(v.x * d.out_scale, v.y * d.out_scale);
      *reinterpret_cast<uint32_t*>(out + off) = pack<P>(v);
    }
    return EPI == 1 ? absmax2(v) : 0.f;
  }
}

// Address tables of a stream step, built once per workgroup with one scatter
// per thread (a lane would otherwise run ~50 serial bit scatters before its
// first load, and scalar scatters of 64-bit values spill scalar registers):
// offsets of every k and n value in A, B and C, of the 16 lane rows in A and
// C, the masks of the row-block bits that count blocks inside an iteration
// (r) and iterations (j), and for each of the four waves the offsets of its
// slot and of its batch index.
//
// Row block numbering inside one batch index (hb = mb - 4 bits, low to high):
// rl bits r (the R blocks of one iteration), wl - bb bits of the wave's slot,
// then the iteration bits; the top bb bits of the wave id select the batch
// index, so a wave's B is fixed.  At each iteration the waves of a batch
// index cover one contiguous window of R * 2^(wl - bb) row blocks, which
// keeps the HBM pages open at any moment few (a contiguous run per wave
// would spread them over the whole tensor).  The r and j parts advance by
// the scattered-bit successor on their masks; C's row bits must be in
// address order like A's (the launcher checks) so the same counters serve.
struct StreamLut {
  uint32_t ak[64], bk[64], bn[64], cn[64];
  uint32_t am[16], cm[16];
  // per wave w: slot offset in A and C, batch offset in A, B and C; then the
  // r and j masks of A and C
  unsigned long long wv[24];
};
enum { WV_XA = 0, WV_XC = 4, WV_AB = 8, WV_BB = 12, WV_CB = 16, WV_MRA = 20, WV_MRC = 21, WV_MJA = 22, WV_MJC = 23 };

// rl = log2 R; iters = 2^(hb + bb - rl - wl) fixes wl.
__device__ __forceinline__ void stream_lut_init(const StepDesc& d, const uint8_t* tab, StreamLut& L, int rl,
                                                uint32_t iters) {
  __syncthreads();  // the position tables copied to tab by every thread
  // One branch-free job shape per wave (divergent branches inside a wave
  // would run one after another): wave 0 the k offsets of A and B, wave 1 the
  // n offsets of B and C, wave 2 the 16 lane rows of A and C, wave 3 the 24
  // per-wave offsets and masks, one bounded scatter per lane.
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int K = 1 << d.kb, N = 1 << d.nb, hb = d.mb - 4;
  const int wl = hb + d.bb - rl - (31 - __builtin_clz(iters));
  const int wlo = wl - d.bb;  // slot bits of the wave id
  if (w == 0) {
    L.ak[l] = (uint32_t)scatter_bits_n<6>(l & (K - 1), tab + T_AK, d.kb);
    L.bk[l] = (uint32_t)scatter_bits_n<6>(l & (K - 1), tab + T_BK, d.kb);
  } else if (w == 1) {
    L.bn[l] = (uint32_t)scatter_bits_n<6>(l & (N - 1), tab + T_BN, d.nb);
    L.cn[l] = (uint32_t)scatter_bits_n<6>(l & (N - 1), tab + T_CN, d.nb);
  } else if (w == 2) {
    if (l < 16) {
      L.am[l] = (uint32_t)scatter_bits_n<4>(l, tab + T_AM, 4);
      L.cm[l] = (uint32_t)scatter_bits_n<4>(l, tab + T_CM, 4);
    }
  } else if (l < 24) {
    // jobs 0-19: (kind, wave) = (l >> 2, l & 3): slot in A, slot in C (the
    // slot fills row-block bits [0, rl + wlo)), batch in A, B, C; jobs 20-23:
    // r and j masks of A and C (row-block bits [0, rl) and [rl + wlo, hb))
    const uint64_t wid = (uint64_t)blockIdx.x * 4 + (l & 3);
    const uint64_t slot = (wid & ((1ull << wlo) - 1)) << rl, batch = wid >> wlo;
    const uint64_t rbits = (1ull << rl) - 1, jbits = ((1ull << hb) - 1) & ~((1ull << (rl + wlo)) - 1);
    const int kind = l >> 2;
    uint64_t x;
    int off, n;
    if (l < 20) {
      x = kind < 2 ? slot : batch;
      off = kind == 0 ? T_AM + 4 : kind == 1 ? T_CM + 4 : kind == 2 ? T_AB : kind == 3 ? T_BB : T_CB;
      n = kind < 2 ? rl + wlo : d.bb;
    } else {
      x = l < 22 ? rbits : jbits;
      off = (l & 1) ? T_CM + 4 : T_AM + 4;
      n = hb;
    }
    L.wv[l] = scatter_bits_n<28>(x, tab + off, n);
  }
  __syncthreads();
}

// x + y recomputed where it is used: the empty volatile asm makes x opaque
// at that point, so the compiler cannot hoist the sum of two loop-invariant
// registers out of the row loop into a third register array (NBLK * KS
// registers that would cost a wave slot per SIMD).  The asm emits no
// instruction; the add stays an ordinary one the compiler schedules (hazard
// checks against the MFMA that reads it included).
__device__ __forceinline__ float add_in_loop(float x, float y) {
  asm volatile("" : "+v"(x));
  return x + y;
}

// A 32-bit lane offset passed through unchanged where it is used, so that
// the compiler keeps it 32 bits wide (hoisted out of the loop it would be
// widened to a 64-bit register pair) and addresses the access as a scalar
// base plus one vector offset register.
__device__ __forceinline__ uint32_t lane_offset(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int P, int KS, int NBLK, int LD, int EPI>
__device__ __forceinline__ float stream_body(const StepDesc& d, const uint8_t* tab, const StreamLut& L,
                                             uint32_t iters) {
  constexpr int R = LD / KS > 0 ? LD / KS : 1;  // row blocks per iteration
  using Raw = typename std::conditional<P == 0, float2, uint32_t>::type;
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const int w = threadIdx.x >> 6;
  const int K = 1 << d.kb, N = 1 << d.nb;
  if (((uint64_t)blockIdx.x * 4 + w) * iters * R >= (1ull << (d.mb - 4 + d.bb)))
    iters = 0;  // a wave past the last row block (grids of one workgroup)
  const uint64_t b_b = L.wv[WV_BB + w];
  // Column group blockIdx.y: this launch's waves cover columns [n0, n0 + 16 NBLK).
  const int n0 = (int)blockIdx.y * 16 * NBLK;
  // MFMA row r of a column block is column n = (r >> 2) + 4 (r & 3) of it, so
  // that output register i of lane group lq is column lq + 4 i: the lowest
  // two n bits sit on lanes and a store instruction covers them.
  // B^T operand: lane holds B[k = 4 ks + lq][n of row lr]
  float br[NBLK][KS], bi[NBLK][KS];
#pragma unroll
  for (int cb = 0; cb < NBLK; ++cb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + lq, n = n0 + 16 * cb + (lr >> 2) + 4 * (lr & 3);
      float2 v = make_float2(0.f, 0.f);
      if (k < K && n < N) v = load_c<P>(d.B, b_b + L.bk[k] + L.bn[n]);
      br[cb][ks] = v.x;
      bi[cb][ks] = v.y;
    }
  // Only K < 4 (one k step) pads inside a k step; the padded lanes read an
  // aliased in-bounds entry and are zeroed.
  const bool kvalid = KS > 1 || lq < K;
  // Lane offsets in bytes, 32 bits (the launcher checks they fit): the four
  // lowest row bits and k = lq (A), n = lq (C).  The rest of k = 4 ks + lq
  // and n = 16 cb + 4 i + lq is the same on every lane: 64-bit scalar
  // offsets added to the scalar base (the offsets of disjoint bits add).
  constexpr uint32_t ESA = sizeof(Raw), ESC = stream_out_bytes<P, EPI>();
  const uint32_t a_lo = (L.am[lr] + L.ak[lq]) * ESA;
  const uint32_t c_lo = (L.cm[lr] + L.cn[lq]) * ESC;
  // (element offsets of at most 2^32-entry tensors: 32-bit scalars)
  uint32_t a_hi[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) a_hi[ks] = __builtin_amdgcn_readfirstlane(L.ak[(4 * ks) & 63]);
  uint32_t c_hb[NBLK], c_hi[4];  // n bits 4-5 (column block) and 2-3
#pragma unroll
  for (int cb = 0; cb < NBLK; ++cb) c_hb[cb] = __builtin_amdgcn_readfirstlane(L.cn[(n0 + 16 * cb) & 63]);
#pragma unroll
  for (int i = 0; i < 4; ++i) c_hi[i] = __builtin_amdgcn_readfirstlane(L.cn[4 * i]);
  // Row-block addresses are wave-uniform: keep them in scalar registers.
  const uint64_t mra = uniform64(L.wv[WV_MRA]), mja = uniform64(L.wv[WV_MJA]), mrc = uniform64(L.wv[WV_MRC]),
                 mjc = uniform64(L.wv[WV_MJC]);
  uint64_t xra = 0, xja = 0, xrc = 0, xjc = 0;
  const char* A = reinterpret_cast<const char*>(d.A) + (uniform64(L.wv[WV_AB + w]) + uniform64(L.wv[WV_XA + w])) * ESA;
  char* out = reinterpret_cast<char*>(EPI == 2 ? (void*)d.acc : d.C) +
              (uniform64(L.wv[WV_CB + w]) + uniform64(L.wv[WV_XC + w])) * ESC;
  float mx = 0.f;
  Raw raw[R][KS];
  auto load = [&](Raw (&dst)[R][KS]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        dst[r][ks] = *reinterpret_cast<const Raw*>(A + ((xra | xja) + (uint64_t)a_hi[ks]) * ESA + lane_offset(a_lo));
      xra = ((xra | ~mra) + 1) & mra;
    }
    xja = ((xja | ~mja) + 1) & mja;
  };
  for (uint32_t it = 0; it < iters; ++it) {
    // All loads of an iteration are issued before any of them is used, so a
    // wave waits for memory once per iteration.
    load(raw);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v4f acc[3][NBLK];
#pragma unroll
      for (int cb = 0; cb < NBLK; ++cb)
#pragma unroll
        for (int p = 0; p < 3; ++p) acc[p][cb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        float2 a;
        if constexpr (P == 0) a = raw[r][ks];
        else a = unpack<P>(raw[r][ks]);
        if (!kvalid) a = make_float2(0.f, 0.f);
        const float as = a.x + a.y;
#pragma unroll
        for (int cb = 0; cb < NBLK; ++cb) {
          acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(br[cb][ks], a.x, acc[0][cb], 0, 0, 0);
          acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bi[cb][ks], a.y, acc[1][cb], 0, 0, 0);
          acc[2][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(add_in_loop(br[cb][ks], bi[cb][ks]), as, acc[2][cb], 0, 0, 0);
        }
      }
      // lane holds C[m = lr][n = 16 cb + lq + 4 i] in register i
#pragma unroll
      for (int cb = 0; cb < NBLK; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (n0 + 16 * cb + lq + 4 * i < N) {
            const float t1 = acc[0][cb][i], t2 = acc[1][cb][i], t3 = acc[2][cb][i];
            mx = fmaxf(mx, stream_store<P, EPI>(out + ((xrc | xjc) + (uint64_t)(c_hb[cb] + c_hi[i])) * ESC, d,
                                                lane_offset(c_lo),
                                                make_float2(t1 - t2, t3 - t1 - t2)));
          }
      xrc = ((xrc | ~mrc) + 1) & mrc;
    }
    xjc = ((xjc | ~mjc) + 1) & mjc;
  }
  return mx;
}

template <int P, int KS, int NBLK, int LD = stream_loads<P>()>
__global__ __launch_bounds__(256) void k_stream(StepDesc d, uint32_t iters) {
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  __shared__ StreamLut lut;
  load_tables(d, tab);
  constexpr int RL = LD / KS > 1 ? ilog2c(LD / KS) : 0;  // log2 R
  stream_lut_init(d, tab, lut, RL, iters);
  float mx;
  if (d.mode == EPI_ACC64) mx = stream_body<P, KS, NBLK, LD, 2>(d, tab, lut, iters);
  else if (d.stats) mx = stream_body<P, KS, NBLK, LD, 1>(d, tab, lut, iters);
  else mx = stream_body<P, KS, NBLK, LD, 0>(d, tab, lut, iters);
  record_max(d, mx);
}

// ---------------------------------------------------------------- stream steps, 16-bit MFMA
// FP16/BF16 storage: the same streaming scheme on the 16 x 16 x 16 FP16/BF16
// MFMA (FP32 accumulate), complex product by the 4M split written as one real
// GEMM: A' = A viewed as the real M x 2K matrix of its interleaved halves
// (the storage itself), B'' = the real 2K x 2N expansion of B with 2 x 2
// blocks [[br, bi], [-bi, br]].  C'^T = B''^T A'^T: one MFMA covers 16 rows m
// (on lanes), 8 complex columns n and 8 complex k.  Lane group lq supplies
// k = 8 ks + 2 lq + {0, 1}: two stored words, as 4 halves, straight from
// HBM.  MFMA row r of a block holds column n = (r >> 2) + 4 ((r >> 1) & 1),
// real (r even) or imaginary part, so output registers (0, 1) and (2, 3) of
// lane group lq are the complex entries n = lq and n = lq + 4.
template <int P, int KS8, int NB8, int EPI>
__device__ __forceinline__ float stream_body_h(const StepDesc& d, const uint8_t* tab, const StreamLut& L,
                                               uint32_t iters) {
  constexpr int R = (1 << kStreamRowsH) / KS8 > 0 ? (1 << kStreamRowsH) / KS8 : 1;  // row blocks per iteration
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const int w = threadIdx.x >> 6;
  const int K = 1 << d.kb, N = 1 << d.nb;
  if (((uint64_t)blockIdx.x * 4 + w) * iters * R >= (1ull << (d.mb - 4 + d.bb)))
    iters = 0;  // a wave past the last row block (grids of one workgroup)
  const uint64_t b_b = L.wv[WV_BB + w];
  // Column group blockIdx.y: this launch's waves cover columns [n0, n0 + 8 NB8).
  const int n0 = (int)blockIdx.y * 8 * NB8;
  // B''^T fragments: row lr of each 16-row block, k' = 4 lq + t
  v4h bf[NB8][KS8];
  {
    const int nl = (lr >> 2) + 4 * ((lr >> 1) & 1), c = lr & 1;
#pragma unroll
    for (int nb = 0; nb < NB8; ++nb)
#pragma unroll
      for (int ks = 0; ks < KS8; ++ks) {
        const int n = n0 + 8 * nb + nl;
        float2 b0 = make_float2(0.f, 0.f), b1 = make_float2(0.f, 0.f);
        const int k0 = 8 * ks + 2 * lq;
        if (n < N && k0 < K) b0 = load_c<P>(d.B, b_b + L.bk[k0] + L.bn[n]);
        if (n < N && k0 + 1 < K) b1 = load_c<P>(d.B, b_b + L.bk[k0 + 1] + L.bn[n]);
        // (c = 0): br, -bi per k; (c = 1): bi, br
        const float e0 = c ? b0.y : b0.x, e1 = c ? b0.x : -b0.y, e2 = c ? b1.y : b1.x, e3 = c ? b1.x : -b1.y;
        bf[nb][ks] = v4h{(_Float16)e0, (_Float16)e1, (_Float16)e2, (_Float16)e3};
        if constexpr (P == 2) {
          // BF16: the same four values as bfloat16 bit patterns
          v4s w{(short)f_to_bf(e0), (short)f_to_bf(e1), (short)f_to_bf(e2), (short)f_to_bf(e3)};
          bf[nb][ks] = __builtin_bit_cast(v4h, w);
        }
      }
  }
  // 32-bit lane offsets hold the four lowest row bits and k = 2 lq + h (A),
  // n = lq (C); the rest of k = 8 ks + 2 lq + h and n = 8 nb + 4 h + lq is
  // wave-uniform and goes to the scalar base, as in stream_body.
  uint32_t a_lo[2];
  bool kv[KS8][2];
#pragma unroll
  for (int h = 0; h < 2; ++h) a_lo[h] = (L.am[lr] + L.ak[2 * lq + h]) * 4u;
#pragma unroll
  for (int ks = 0; ks < KS8; ++ks)
#pragma unroll
    for (int h = 0; h < 2; ++h) kv[ks][h] = 8 * ks + 2 * lq + h < K;
  uint32_t a_hi[KS8];
#pragma unroll
  for (int ks = 0; ks < KS8; ++ks) a_hi[ks] = __builtin_amdgcn_readfirstlane(L.ak[(8 * ks) & 63]);
  constexpr uint32_t ESC = stream_out_bytes<P, EPI>();
  const uint32_t c_lo = (L.cm[lr] + L.cn[lq]) * ESC;
  uint32_t c_hb[NB8];  // n bits 3-5 (column block); bit 2 is h
#pragma unroll
  for (int nb = 0; nb < NB8; ++nb) c_hb[nb] = __builtin_amdgcn_readfirstlane(L.cn[(n0 + 8 * nb) & 63]);
  const uint32_t c_h4 = __builtin_amdgcn_readfirstlane(L.cn[4]);
  const uint64_t mra = uniform64(L.wv[WV_MRA]), mja = uniform64(L.wv[WV_MJA]), mrc = uniform64(L.wv[WV_MRC]),
                 mjc = uniform64(L.wv[WV_MJC]);
  uint64_t xra = 0, xja = 0, xrc = 0, xjc = 0;
  const char* A = reinterpret_cast<const char*>(d.A) + (uniform64(L.wv[WV_AB + w]) + uniform64(L.wv[WV_XA + w])) * 4u;
  char* out = reinterpret_cast<char*>(EPI == 2 ? (void*)d.acc : d.C) +
              (uniform64(L.wv[WV_CB + w]) + uniform64(L.wv[WV_XC + w])) * ESC;
  float mx = 0.f;
  for (uint32_t it = 0; it < iters; ++it) {
    uint32_t raw[R][KS8][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int ks = 0; ks < KS8; ++ks)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          raw[r][ks][h] =
              *reinterpret_cast<const uint32_t*>(A + ((xra | xja) + (uint64_t)a_hi[ks]) * 4u + lane_offset(a_lo[h]));
      xra = ((xra | ~mra) + 1) & mra;
    }
    xja = ((xja | ~mja) + 1) & mja;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v4f acc[NB8];
#pragma unroll
      for (int nb = 0; nb < NB8; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS8; ++ks) {
        const uint32_t w0 = kv[ks][0] ? raw[r][ks][0] : 0u, w1 = kv[ks][1] ? raw[r][ks][1] : 0u;
        const v4h a = __builtin_bit_cast(v4h, (uint64_t)w0 | ((uint64_t)w1 << 32));
#pragma unroll
        for (int nb = 0; nb < NB8; ++nb) {
          if constexpr (P == 1) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16f16(bf[nb][ks], a, acc[nb], 0, 0, 0);
          else
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, bf[nb][ks]),
                                                                __builtin_bit_cast(v4s, a), acc[nb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int nb = 0; nb < NB8; ++nb)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (n0 + 8 * nb + lq + 4 * h < N)
            mx = fmaxf(mx, stream_store<P, EPI>(out + ((xrc | xjc) + (uint64_t)(c_hb[nb] + (h ? c_h4 : 0u))) * ESC, d,
                                                lane_offset(c_lo),
                                                make_float2(acc[nb][2 * h], acc[nb][2 * h + 1])));
      xrc = ((xrc | ~mrc) + 1) & mrc;
    }
    xjc = ((xjc | ~mjc) + 1) & mjc;
  }
  return mx;
}

template <int P, int KS8, int NB8>
__global__ __launch_bounds__(256) void k_stream_h(StepDesc d, uint32_t iters) {
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  __shared__ StreamLut lut;
  load_tables(d, tab);
  constexpr int RL = kStreamRowsH > ilog2c(KS8) ? kStreamRowsH - ilog2c(KS8) : 0;  // log2 R
  stream_lut_init(d, tab, lut, RL, iters);
  float mx;
  if (d.mode == EPI_ACC64) mx = stream_body_h<P, KS8, NB8, 2>(d, tab, lut, iters);
  else if (d.stats) mx = stream_body_h<P, KS8, NB8, 1>(d, tab, lut, iters);
  else mx = stream_body_h<P, KS8, NB8, 0>(d, tab, lut, iters);
  record_max(d, mx);
}

// ---------------------------------------------------------------- fused stem sections
// A chain of stream-like steps on one large tensor T run in one kernel
// (Sec. IV: the stem tensor stays on chip while small tensors are absorbed;
// a section of n steps saves 2 (n - 1) passes over T).  Each workgroup takes
// tiles of T in turn: it loads the tile (every bit the section contracts,
// plus low address bits, enumerated in A's address order so the loads are
// coalesced) into an LDS buffer, applies the steps between two LDS buffers
// and writes the final tile in C's address order.  Inside a step the MFMA
// mapping is the stream kernel's (C^T = B^T A^T, 3M split), with A read from
// LDS and each step's padded B^T kept in LDS for the whole kernel.

// Deposits the low n bits of x at the bits pos[0..n) (n <= 16); pos is a
// 4-byte aligned byte table in LDS, read a word at a time.
__device__ __forceinline__ uint32_t scatter16(uint32_t x, const uint8_t* pos, int n) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(pos);
  uint32_t r = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (4 * q < n) {
      const uint32_t word = w[q];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (4 * q + b < n) r |= ((x >> (4 * q + b)) & 1u) << ((word >> (8 * b)) & 31u);
    }
  }
  return r;
}

static_assert(offsetof(TileStep, am) % 4 == 0 && offsetof(TileStep, ak) % 4 == 0 && offsetof(TileStep, cm) % 4 == 0 &&
                  offsetof(TileStep, cn) % 4 == 0 && offsetof(TileStep, bk) % 4 == 0 &&
                  offsetof(TileStep, bn) % 4 == 0 && sizeof(TileStep) % 8 == 0,
              "tile-step tables must be word aligned");
static_assert(offsetof(SectionDesc, p_in) % 4 == 0 && offsetof(SectionDesc, p_out) % 4 == 0 &&
                  offsetof(SectionDesc, st) % 8 == 0 && sizeof(SectionDesc) % 4 == 0,
              "section tables must be word aligned");

__device__ __forceinline__ void record_max_at(float* stats, int idx, float m) {
  __shared__ float red[16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
    if (m > 0.f) raise_max(reinterpret_cast<unsigned int*>(stats) + idx, m);
  }
}

// A byte table in LDS (4-byte aligned) read as NW wave-uniform words, so
// that scatters of wave-uniform values through it are scalar work.
template <int NW>
struct UTab {
  uint32_t w[NW];
  __device__ __forceinline__ explicit UTab(const uint8_t* p) {
#pragma unroll
    for (int q = 0; q < NW; ++q) w[q] = __builtin_amdgcn_readfirstlane(reinterpret_cast<const uint32_t*>(p)[q]);
  }
  __device__ __forceinline__ uint32_t pos(int i) const { return (w[i >> 2] >> (8 * (i & 3))) & 31u; }
  // deposits bit i of x at pos(first + i), i < n (first + n <= 4 NW)
  __device__ __forceinline__ uint32_t scatter(uint32_t x, int first, int n) const {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 4 * NW; ++i)
      if (i >= first && i < first + n) r |= ((x >> (i - first)) & 1u) << pos(i);
    return r;
  }
};

// One step of a section on LDS-resident tiles (KS k steps of 4, NBLK column
// blocks of 16, as in the stream kernel); returns the largest stored
// magnitude of this thread when `want_max`.
template <int KS, int NBLK>
__device__ __forceinline__ float section_step_t(const TileStep& ts, const float2* in, float2* out, const float2* Bl,
                                                bool want_max, int tb_bits, int stride_bits) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nwaves = blockDim.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int kb = __builtin_amdgcn_readfirstlane(ts.kb), nb = __builtin_amdgcn_readfirstlane(ts.nb);
  const int mb = __builtin_amdgcn_readfirstlane(ts.mb);
  const uint32_t kpad = __builtin_amdgcn_readfirstlane(ts.kpad), b_lds = __builtin_amdgcn_readfirstlane(ts.b_lds);
  const float osc = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, ts.out_scale)));
  const int K = 1 << kb, N = 1 << nb;
  const bool kvalid = KS > 1 || lq < K;
  const UTab<4> am(ts.am), cm(ts.cm);
  const UTab<2> ak(ts.ak), cn(ts.cn);
  // B fragments in registers: column (lr >> 2) + 4 (lr & 3) of column block
  // cb; LDS holds B as [cb][k][16 columns] (64 consecutive entries per read)
  float br[NBLK][KS], bi[NBLK][KS], bs[NBLK][KS];
  const uint32_t b_lane = b_lds + (uint32_t)lq * 16 + (uint32_t)((lr >> 2) + 4 * (lr & 3));
#pragma unroll
  for (int cb = 0; cb < NBLK; ++cb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float2 b = Bl[b_lane + ((uint32_t)cb * kpad + 4 * ks) * 16];
      br[cb][ks] = b.x;
      bi[cb][ks] = b.y;
      bs[cb][ks] = b.x + b.y;
    }
  // lane parts (4 rows bits, 2 k bits, 2 n bits) plus scalar parts
  const int kl = kb < 2 ? kb : 2, nl = nb < 2 ? nb : 2;
  const uint32_t a_lane = am.scatter(lr, 0, 4) + ak.scatter(lq, 0, kl);
  const uint32_t c_lane = cm.scatter(lr, 0, 4) + cn.scatter(lq, 0, nl);
  uint32_t a_k[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) a_k[ks] = a_lane + ak.scatter(ks, 2, kb - kl);
  uint32_t c_n[NBLK][4];
#pragma unroll
  for (int cb = 0; cb < NBLK; ++cb)
#pragma unroll
    for (int i = 0; i < 4; ++i) c_n[cb][i] = c_lane + cn.scatter(i + 4 * cb, 2, nb - nl);
  const int hb = mb - 4;
  const int nblk = 1 << (hb + tb_bits);  // row blocks of every tile of the group
  float mx = 0.f;
  for (int blk = wave; blk < nblk; blk += nwaves) {
    const uint32_t tslot = (uint32_t)(blk >> hb) << stride_bits;
    const uint32_t xa = tslot + am.scatter(blk, 4, hb), xc = tslot + cm.scatter(blk, 4, hb);
    float2 av[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) av[ks] = in[xa + a_k[ks]];
    v4f acc[3][NBLK];
#pragma unroll
    for (int cb = 0; cb < NBLK; ++cb)
#pragma unroll
      for (int p = 0; p < 3; ++p) acc[p][cb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      float2 a = av[ks];
      if (!kvalid) a = make_float2(0.f, 0.f);
      const float as = a.x + a.y;
#pragma unroll
      for (int cb = 0; cb < NBLK; ++cb) {
        acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(br[cb][ks], a.x, acc[0][cb], 0, 0, 0);
        acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bi[cb][ks], a.y, acc[1][cb], 0, 0, 0);
        acc[2][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bs[cb][ks], as, acc[2][cb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < NBLK; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (16 * cb + lq + 4 * i < N) {
          const float t1 = acc[0][cb][i], t2 = acc[1][cb][i], t3 = acc[2][cb][i];
          const float2 v = make_float2((t1 - t2) * osc, (t3 - t1 - t2) * osc);
          out[xc + c_n[cb][i]] = v;
          if (want_max) mx = fmaxf(mx, absmax2(v));
        }
  }
  return mx;
}

__device__ __forceinline__ float section_step(const TileStep& ts, const float2* in, float2* out, const float2* Bl,
                                              bool want_max, int tb_bits, int stride_bits) {
  const int kb = __builtin_amdgcn_readfirstlane(ts.kb), nb = __builtin_amdgcn_readfirstlane(ts.nb);
  const int ksl = kb > 2 ? kb - 2 : 0, nbl = nb > 4 ? nb - 4 : 0;
#define MITNC_SEC(KSL, NBL) \
  if (ksl == KSL && nbl == NBL) return section_step_t<1 << KSL, 1 << NBL>(ts, in, out, Bl, want_max, tb_bits, stride_bits);
  MITNC_SEC(0, 0) MITNC_SEC(1, 0) MITNC_SEC(2, 0) MITNC_SEC(3, 0) MITNC_SEC(4, 0)
  MITNC_SEC(0, 1) MITNC_SEC(1, 1) MITNC_SEC(2, 1) MITNC_SEC(3, 1)
  MITNC_SEC(0, 2) MITNC_SEC(1, 2) MITNC_SEC(2, 2)
#undef MITNC_SEC
  return 0.f;  // not reached: the planner keeps K N within these
}

template <int P>
__global__ __launch_bounds__(256) void k_section(SectionDesc sd_arg) {
  extern __shared__ float2 dyn[];
  // Tables are read from an LDS copy (a dynamically indexed kernel argument
  // would be copied to scratch); global pointers come from the argument
  // itself (a pointer read back from LDS is generic, and generic accesses
  // also count against the LDS wait counter).
  __shared__ SectionDesc sd;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&sd_arg);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&sd);
    for (int i = threadIdx.x; i < (int)(sizeof(SectionDesc) / 4); i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const int tile_max = __builtin_amdgcn_readfirstlane(sd.tile_max);
  const int n_steps = __builtin_amdgcn_readfirstlane(sd.n_steps);
  const int t_in = __builtin_amdgcn_readfirstlane(sd.t_in), t_out = __builtin_amdgcn_readfirstlane(sd.t_out);
  const int outer_bits = __builtin_amdgcn_readfirstlane(sd.outer_bits);
  float2* buf0 = dyn;
  float2* buf1 = dyn + tile_max;
  float2* Bl = dyn + 2 * tile_max;
  const int tid = threadIdx.x;
  // padded B of every step as [column block][k (kpad)][16 columns], zero
  // outside K x N
#pragma unroll
  for (int j = 0; j < kMaxSectionSteps; ++j) {
    if (j < n_steps) {
      const TileStep& ts = sd.st[j];
      const void* Bp = sd_arg.st[j].B;
      const int K = 1 << ts.kb, N = 1 << ts.nb;
      const int rows = N > 16 ? N : 16;
      const UTab<2> bk(ts.bk), bn(ts.bn);
      for (int idx = tid; idx < rows * (int)ts.kpad; idx += blockDim.x) {
        const int c = idx & 15, k = (idx >> 4) % ts.kpad, n = (idx >> 4) / ts.kpad * 16 + c;
        float2 v = make_float2(0.f, 0.f);
        if (k < K && n < N) v = load_c<P>(Bp, bk.scatter(k, 0, ts.kb) + bn.scatter(n, 0, ts.nb));
        Bl[ts.b_lds + idx] = v;
      }
    }
  }
  __syncthreads();
  const UTab<4> pin(sd.p_in), pout(sd.p_out);
  const UTab<8> qin(sd.q_in), qout(sd.q_out);
  // element e = tid + 256 u of a tile: low 8 bits from tid, the rest uniform
  const uint32_t lo_in = pin.scatter(tid, 0, 8), lo_out = pout.scatter(tid, 0, 8);
  const int hi_in = 1 << (t_in - 8), hi_out = 1 << (t_out - 8);
  auto outer_off = [](const UTab<8>& q, uint64_t tile, int n) {
    uint64_t r = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i)
      if (i < n) r |= ((tile >> i) & 1ull) << q.pos(i);
    return r;
  };
  float smx[kMaxSectionSteps];
#pragma unroll
  for (int j = 0; j < kMaxSectionSteps; ++j) smx[j] = 0.f;
  const int tb_bits = __builtin_amdgcn_readfirstlane(sd.tb_bits);
  const int stride_bits = __builtin_amdgcn_readfirstlane(sd.stride_bits);
  // Tiles go in groups of 2^tb_bits; element E = tid + 256 u of a group is
  // entry E mod 2^t of tile E >> t (t >= 8, so the tile index is uniform),
  // stored at slot (tile << stride_bits) of a buffer.
  const uint64_t n_groups = 1ull << (outer_bits - tb_bits);
  const int n_in = 1 << (t_in + tb_bits - 8), n_out = 1 << (t_out + tb_bits - 8);  // <= 16 each
  float2 pre[16];
  uint64_t grp = blockIdx.x;
  if (grp < n_groups) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int uu = u < n_in ? u : 0;  // past the group: entry 0 again, in bounds, not kept
      const int t = uu >> (t_in - 8);
      const uint64_t oin = outer_off(qin, (grp << tb_bits) + t, outer_bits);
      pre[u] = load_c<P>(sd_arg.A, oin + lo_in + pin.scatter((uint32_t)uu, 8, t_in - 8));
    }
  }
  for (; grp < n_groups; grp += gridDim.x) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (u < n_in) {
        const int t = u >> (t_in - 8);
        buf0[((uint32_t)t << stride_bits) + tid + 256 * (u & ((1 << (t_in - 8)) - 1))] = pre[u];
      }
    __syncthreads();
    if (grp + gridDim.x < n_groups) {
      const uint64_t nxt = grp + gridDim.x;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int uu = u < n_in ? u : 0;
        const int t = uu >> (t_in - 8);
        const uint64_t oin = outer_off(qin, (nxt << tb_bits) + t, outer_bits);
        pre[u] = load_c<P>(sd_arg.A, oin + lo_in + pin.scatter((uint32_t)uu, 8, t_in - 8));
      }
    }
    for (int j = 0; j < n_steps; ++j) {
      smx[j & 7] = fmaxf(smx[j & 7], section_step(sd.st[j], (j & 1) ? buf1 : buf0, (j & 1) ? buf0 : buf1, Bl,
                                                  sd_arg.stats != nullptr, tb_bits, stride_bits));
      __syncthreads();
    }
    const float2* fin = (n_steps & 1) ? buf1 : buf0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (u < n_out) {
        const int t = u >> (t_out - 8);
        const uint64_t oout = outer_off(qout, (grp << tb_bits) + t, outer_bits);
        const uint32_t hi = pout.scatter((uint32_t)u, 8, t_out - 8);
        const float2 v = fin[((uint32_t)t << stride_bits) + tid + 256 * (u & ((1 << (t_out - 8)) - 1))];
        if constexpr (P == 0) reinterpret_cast<float2*>(sd_arg.C)[oout + lo_out + hi] = v;
        else reinterpret_cast<uint32_t*>(sd_arg.C)[oout + lo_out + hi] = pack<P>(v);
      }
    }
    __syncthreads();
  }
  if (sd_arg.stats) {
    for (int j = 0; j < n_steps; ++j) {
      record_max_at(sd_arg.stats, sd.st[j].step_index, smx[j & 7]);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- tile helpers
// Decodes a tile element number into its logical coordinates and address
// offset; codes/tables live in LDS.
struct TileSlot {
  uint32_t off;
  int lo, hi;  // (m, k) for A tiles, (k, n) for B tiles, (m, n) for C tiles
};

// Tile bits [B0, B1) of element number e (the others are ignored); the
// decode of e is the OR of the decodes of disjoint bit ranges, so a thread
// decodes the bits its thread index gives once and adds the bits of each
// load slot (uniform across the workgroup) separately.  Unrolled so that the
// LDS reads of one decode are independent of each other (two round trips
// instead of two per bit).
template <int B0, int B1>
__device__ __forceinline__ TileSlot decode_bits(uint32_t e, int nbits, const uint8_t* codes, const uint8_t* tab,
                                                int first_cls, int off_first, int off_second) {
  // Branch-free (index clamped, contribution masked): the LDS reads of all
  // bits issue together instead of one dependent pair per bit.  Both
  // position tables are read and the one of the bit's class kept by masks,
  // so no control flow or scalar select depends on the class.
  TileSlot r{0, 0, 0};
#pragma unroll
  for (int b = B0; b < B1; ++b) {
    const int on = b < nbits ? 1 : 0;
    const int code = codes[on ? b : 0];
    const int idx = code & 31;
    const int m = (((code >> 5) ^ first_cls) - 1) >> 31;  // all ones for the first class
    const int pos = (tab[off_first + idx] & m) | (tab[off_second + idx] & ~m);
    const int bit = (e >> b) & on;
    r.lo |= (bit << idx) & m;
    r.hi |= (bit << idx) & ~m;
    r.off |= (uint32_t)bit << pos;
  }
  return r;
}

__device__ __forceinline__ TileSlot or_slots(TileSlot a, TileSlot b) {
  return TileSlot{a.off | b.off, a.lo | b.lo, a.hi | b.hi};
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Stores the staged C tile (LDS, complex float, row stride SC) to the output,
// enumerating the tile in C's address order; WK partial tiles are summed.
template <int P, int TM, int WK, int SC, int C_ITEMS>
__device__ __forceinline__ void store_c_tile(const StepDesc& d, const uint8_t* tab, const float2* Cs, uint64_t mt,
                                             uint64_t nt, uint64_t batch) {
  const int tid = threadIdx.x;
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  const uint64_t baseC = wave_scatter(mt, tab + T_CM + d.tm, d.mb - d.tm) +
                         wave_scatter(nt, tab + T_CN + d.tn, d.nb - d.tn) + wave_scatter(batch, tab + T_CB, d.bb);
  const int nc = d.tm + d.tn;
  // Element e = tid + 256 j: the low 8 tile bits come from tid (decoded once
  // per thread), the others from j (uniform across the workgroup).
  const int nlo = nc < 8 ? nc : 8;
  const bool active = tid < (1 << nlo);
  const TileSlot lo = decode_bits<0, 8>(tid & ((1 << nlo) - 1), nlo, tab + T_CTILE, tab, TB_M, T_CM, T_CN);
  const int n_hi = 1 << (nc - nlo);
  // The high parts are uniform: item j is the OR of the decodes of its set
  // bits (tile bits 8 + t, t < log2 C_ITEMS), each decoded once into
  // wave-uniform registers, so an item's LDS address is the thread's part
  // plus a uniform offset and all items' LDS reads issue back to back.
  constexpr int HB = ilog2(C_ITEMS);
  uint32_t h_off[HB > 0 ? HB : 1];
  int h_lds[HB > 0 ? HB : 1];
#pragma unroll
  for (int t = 0; t < HB; ++t) {
    const TileSlot h = decode_bits<8, 16>(1u << (8 + t), nc, tab + T_CTILE, tab, TB_M, T_CM, T_CN);
    h_off[t] = __builtin_amdgcn_readfirstlane(h.off);
    h_lds[t] = __builtin_amdgcn_readfirstlane(h.lo * SC + h.hi);  // disjoint bits: OR = sum
  }
  const int lds_lo = lo.lo * SC + lo.hi;
  float2 vals[C_ITEMS];
#pragma unroll
  for (int j = 0; j < C_ITEMS; ++j) {
    int hl = 0;
#pragma unroll
    for (int t = 0; t < HB; ++t)
      if ((j >> t) & 1) hl += h_lds[t];
    float2 v = make_float2(0.f, 0.f);
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      const float2 c = Cs[w * TM * SC + lds_lo + hl];
      v.x += c.x;
      v.y += c.y;
    }
    vals[j] = v;
  }
  float mx = 0.f;
#pragma unroll
  for (int j = 0; j < C_ITEMS; ++j) {
    uint32_t ho = 0;
#pragma unroll
    for (int t = 0; t < HB; ++t)
      if ((j >> t) & 1) ho |= h_off[t];
    if (active && j < n_hi) mx = fmaxf(mx, epilogue_store<P>(d, baseC + (lo.off | ho), vals[j], blockIdx.y, c_elems));
  }
  record_max(d, mx);
}

// ---------------------------------------------------------------- FP32 MFMA tiles
// Workgroup of 4 waves computes a TM x TN complex tile of C over a range of
// TK-wide k tiles.  WM x WN x WK waves: WM x WN split the tile, WK split each
// k tile (their partial tiles are summed in LDS in a fixed order).
//
// Global -> LDS: each thread owns fixed tile elements enumerated in the
// operand's address order (coalesced), and writes them to the LDS position of
// their logical (m, k) / (k, n) coordinate: the permutation happens here
// (Sec. V-A, in-kernel permutation; on a SIMT machine the shuffle is the
// scattered LDS write).  LDS holds two stages, so one barrier per k tile
// suffices and the next tile's global loads overlap the MFMAs.
//
// Complex product by the 3M split: T1 = Ar Br, T2 = Ai Bi,
// T3 = (Ar + Ai)(Br + Bi), Re C = T1 - T2, Im C = T3 - T1 - T2: three real
// 16 x 16 x 4 FP32 MFMAs per 16 x 16 complex block and 4 complex k, instead of
// the four of the 4M split.
// Column XOR of LDS row k of a complex64 tile operand: the XOR of swz[j]
// over the set bits j of k, kept inside the row (mask = columns - 1).
__device__ __forceinline__ int row_xor(const uint8_t* swz, int k, int mask) {
  int h = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) h ^= ((k >> j) & 1) ? (int)swz[j] : 0;
  return h & mask;
}

// Output tile (mt, nt) of tile index x among n_mt x n_nt tiles.  Workgroups
// are dealt round-robin over the 8 XCDs, each with its own L2, and the
// kernels take tile indices x = workgroup + i * (multiple of 8), so x & 7 is
// the XCD.  An XCD owns the m blocks mt = 8 r + xcd and walks its (r, nt)
// tiles in groups of up to 8 consecutive r: inside a group r is the fastest
// index, so the ~64 tiles an XCD holds at once span about 8 m blocks by 8 n
// blocks.  At each k stage they then read about 8 A and 8 B stage tiles
// instead of 64 A tiles and one B tile (m fastest over the whole grid), so
// far fewer operand tiles miss in L2.
__device__ __forceinline__ void tile_of(uint64_t x, uint64_t n_mt, uint64_t n_nt, uint64_t& mt, uint64_t& nt) {
  if ((n_mt & 7) == 0 && n_nt > 1) {
    const uint64_t i = x >> 3, nm = n_mt >> 3;
    const uint64_t gm = nm < 8 ? nm : 8;
    const uint64_t grp = i / (gm * n_nt), within = i % (gm * n_nt);
    mt = ((grp * gm + within % gm) << 3) | (x & 7);
    nt = within / gm;
  } else {
    mt = x % n_mt;
    nt = x / n_mt;
  }
}

template <int WM, int WN, int WK, int BM, int BN, int TK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_tile(StepDesc d) {
  constexpr int TM = WM * BM * 16;
  constexpr int TN = WN * BN * 16;
  constexpr int KW = TK / WK;                   // complex k per wave and k tile
  static_assert(KW % 4 == 0, "k per wave must be a multiple of 4");
  // LDS rows of A and B are the k of the tile, unpadded: row k stores column
  // c at c ^ H(k), with the step's row masks (StepDesc::a_swz, b_swz).
  constexpr int SA = TM;                        // float2 per LDS row of A (row = k)
  constexpr int SB = TN;                        // float2 per LDS row of B (row = k)
  constexpr int STAGE = TK * SA + TK * SB;      // float2 per stage
  constexpr int SC = TN + 4;                    // float2 per LDS row of the C tile
  constexpr int A_LOADS = TM * TK / 256;
  constexpr int B_LOADS = (TK * TN + 255) / 256;
  constexpr int C_ITEMS = TM * TN / 256;
  constexpr int SMEM_AB = 2 * STAGE;
  constexpr int SMEM_C = WK * TM * SC;
  constexpr int SMEM = SMEM_AB > SMEM_C ? SMEM_AB : SMEM_C;
  static_assert(A_LOADS >= 1 && C_ITEMS >= 1, "tile too small");
  __shared__ float2 smem[SMEM];
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  __shared__ uint64_t flip[2][32];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = (wave / WM) % WN, wk = wave / (WM * WN);
  const float2* A = reinterpret_cast<const float2*>(d.A);
  const float2* B = reinterpret_cast<const float2*>(d.B);

  load_tables(d, tab);
  __syncthreads();
  // Padded k (fewer k bits than the stage) must read as zero in both
  // operands; other entries outside the valid tile only feed outputs that
  // are never stored.  A tile's C staging overwrites the stages, so with
  // padded k the stages are zeroed again for every tile.
  const bool pad_k = d.tk < __builtin_ctz(TK);
  uint64_t baseA = 0, baseB = 0;  // tile origins in A and B (set per output tile)

  // Per-thread load slots: global offset inside the tile and LDS index.
  // Decoding ignores bits at or above the operand's tile bits, so a slot
  // past a tile smaller than the template repeats a valid one (same load,
  // same value to the same LDS slot): loads and stores need no branches.
  // Slot tid + 256 j: the low 8 tile bits come from tid, the others from j.
  static_assert((A_LOADS & (A_LOADS - 1)) == 0 && (B_LOADS & (B_LOADS - 1)) == 0, "load counts are powers of two");
  uint32_t a_off[A_LOADS];
  int a_lds[A_LOADS];
  const int na = d.tm + d.tk;
  const TileSlot a_base = decode_bits<0, 8>(tid, na, tab + T_ATILE, tab, TB_M, T_AM, T_AK);
#pragma unroll
  for (int j = 0; j < A_LOADS; ++j) {
    const TileSlot s =
        or_slots(a_base, decode_bits<8, 8 + ilog2(A_LOADS)>(256u * j, na, tab + T_ATILE, tab, TB_M, T_AM, T_AK));
    a_off[j] = s.off;
    a_lds[j] = s.hi * SA + (s.lo ^ row_xor(d.a_swz, s.hi, TM - 1));
  }
  uint32_t b_off[B_LOADS];
  int b_lds[B_LOADS];
  const int nbt = d.tk + d.tn;
  const TileSlot b_base = decode_bits<0, 8>(tid, nbt, tab + T_BTILE, tab, TB_K, T_BK, T_BN);
#pragma unroll
  for (int j = 0; j < B_LOADS; ++j) {
    const TileSlot s =
        or_slots(b_base, decode_bits<8, 8 + ilog2(B_LOADS)>(256u * j, nbt, tab + T_BTILE, tab, TB_K, T_BK, T_BN));
    b_off[j] = s.off;
    b_lds[j] = TK * SA + s.lo * SB + (s.hi ^ row_xor(d.b_swz, s.lo, TN - 1));
  }

  const uint64_t k_tiles = 1ull << (d.kb - d.tk);
  const uint64_t per = k_tiles >> d.ks_bits;
  const uint64_t kt0 = (uint64_t)blockIdx.y * per;
  const int khb = d.kb - d.tk;
  // Address offsets of the current k tile in A and B.  Going from k tile t
  // to t + 1 flips the logical high-k bits 0 .. ctz(t + 1); flip[.][j] holds
  // the address bits of logical bits 0 .. j, so each step is one XOR.
  if (tid < khb) {
    uint64_t fa = 0, fb = 0;
    for (int i = 0; i <= tid; ++i) {
      fa |= 1ull << tab[T_AK + d.tk + i];
      fb |= 1ull << tab[T_BK + d.tk + i];
    }
    flip[0][tid] = fa;
    flip[1][tid] = fb;
  }
  const uint64_t ka0 = wave_scatter(kt0, tab + T_AK + d.tk, khb);
  const uint64_t kbo0 = wave_scatter(kt0, tab + T_BK + d.tk, khb);
  uint64_t ka = ka0, kbo = kbo0;

  // Two register sets of staged loads: k tile t + 2 is requested while
  // tile t is computed and tile t + 1 (requested one tile earlier) goes to
  // the other LDS stage, so every load has two tiles of MFMA work to land.
  float2 ra[2][A_LOADS], rb[2][B_LOADS];
  auto load = [&](int r) {
#pragma unroll
    for (int j = 0; j < A_LOADS; ++j) ra[r][j] = A[baseA + ka + a_off[j]];
#pragma unroll
    for (int j = 0; j < B_LOADS; ++j) rb[r][j] = B[baseB + kbo + b_off[j]];
  };
  auto store = [&](int r, int stage) {
    float2* S = smem + stage * STAGE;
#pragma unroll
    for (int j = 0; j < A_LOADS; ++j) S[a_lds[j]] = ra[r][j];
#pragma unroll
    for (int j = 0; j < B_LOADS; ++j) S[b_lds[j]] = rb[r][j];
  };
  // Moves the load offsets from k tile kt0 + t - 1 to kt0 + t (t >= 1).
  auto advance = [&](uint64_t t) {
    const int fl = __builtin_ctzll(kt0 + t);
    ka ^= flip[0][fl];
    kbo ^= flip[1][fl];
  };

  v4f acc[3][BM][BN];
  const int row = lane & 15, kq = lane >> 4;
  auto compute = [&](int cur) {
    const float2* As = smem + cur * STAGE;
    const float2* Bs = As + TK * SA;
    float2 av[KW / 4][BM], bv[KW / 4][BN];
#pragma unroll
    for (int ks = 0; ks < KW / 4; ++ks) {
      const int k = wk * KW + ks * 4 + kq;
      const int ha = row_xor(d.a_swz, k, TM - 1), hb = row_xor(d.b_swz, k, TN - 1);
#pragma unroll
      for (int bm = 0; bm < BM; ++bm) av[ks][bm] = As[k * SA + (((wm * BM + bm) * 16 + row) ^ ha)];
#pragma unroll
      for (int bn = 0; bn < BN; ++bn) bv[ks][bn] = Bs[k * SB + (((wn * BN + bn) * 16 + row) ^ hb)];
    }
#pragma unroll
    for (int ks = 0; ks < KW / 4; ++ks)
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn) {
          const float2 a = av[ks][bm], b = bv[ks][bn];
          acc[0][bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[0][bm][bn], 0, 0, 0);
          acc[1][bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[1][bm][bn], 0, 0, 0);
          acc[2][bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, b.x + b.y, acc[2][bm][bn], 0, 0, 0);
        }
  };
  // One k tile: stage it & 1 holds tile it, register set x holds tile it + 1.
  auto step = [&](uint64_t it, int x) {
    if (it + 2 < per) {
      advance(it + 2);
      load(x ^ 1);
    }
    compute((int)(it & 1));
    if (it + 1 < per) store(x, (int)(it & 1) ^ 1);
    __syncthreads();
  };

  __syncthreads();  // flip[][] (written above by threads tid < khb) is read from here on
  // Output tiles are dealt grid-stride (the launch holds about as many
  // workgroups as are resident), so the set-up above is paid once per
  // workgroup and a tile's stores drain while the next tile loads.
  const uint64_t n_mt = 1ull << (d.mb - d.tm), n_nt = 1ull << (d.nb - d.tn);
  const uint64_t batch = blockIdx.z;
  for (uint64_t tx = blockIdx.x; tx < n_mt * n_nt; tx += gridDim.x) {
    uint64_t mt, nt;
    tile_of(tx, n_mt, n_nt, mt, nt);
    baseA = wave_scatter(mt, tab + T_AM + d.tm, d.mb - d.tm) + wave_scatter(batch, tab + T_AB, d.bb);
    baseB = wave_scatter(nt, tab + T_BN + d.tn, d.nb - d.tn) + wave_scatter(batch, tab + T_BB, d.bb);
    ka = ka0;
    kbo = kbo0;
    if (pad_k) {
      for (int i = tid; i < SMEM_AB; i += 256) smem[i] = make_float2(0.f, 0.f);
      __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[p][i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    load(0);
    if (per > 1) {
      advance(1);
      load(1);
    }
    store(0, 0);
    __syncthreads();
    for (uint64_t it = 0; it < per; it += 2) {
      step(it, 1);
      if (it + 1 < per) step(it + 1, 0);
    }
    // Accumulators -> LDS tile: Re = T1 - T2, Im = T3 - T1 - T2.
    float2* Cs = smem;
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = (wm * BM + bm) * 16 + 4 * kq + i;
          const int n = (wn * BN + bn) * 16 + row;
          const float t1 = acc[0][bm][bn][i], t2 = acc[1][bm][bn][i], t3 = acc[2][bm][bn][i];
          Cs[(wk * TM + m) * SC + n] = make_float2(t1 - t2, t3 - t1 - t2);
        }
    __syncthreads();
    store_c_tile<0, TM, WK, SC, C_ITEMS>(d, tab, Cs, mt, nt, batch);
    __syncthreads();  // the next tile's staging overwrites the C tile
  }
}

// ---------------------------------------------------------------- FP16 / BF16 MFMA tiles
// Same structure with 16-bit storage and the 4M split on the 16 x 16 x 32
// FP16/BF16 MFMA (FP32 accumulate): A is viewed as the real M x 2K matrix
// A'[m][2k + p] = (Re, Im)[p] of A[m][k] -- exactly the interleaved storage --
// and B is expanded in LDS into 2 x 2 real blocks [[br, bi], [-bi, br]]
// (rows 2k, 2k+1; columns 2n, 2n+1), so A' B' holds Re C in even and Im C in
// odd columns.  One MFMA covers 16 rows, 8 complex columns and 16 complex k.
// LDS rows hold one complex k per 32-bit word: A row m holds A[m][k], B'
// row 2n + c holds the words (br, -bi) (c = 0) or (bi, br) (c = 1) of
// B[k][n].  Word addresses follow the step's GF(2)-linear map (StepDesc::
// ha_row, hb_row, hk): the order of the k inside a row is the same for A and
// B (the sum over k does not depend on it) and 4-word groups are permuted
// per row so that staging writes and fragment reads spread over the banks.

// XOR of rows[i] over the set bits i of r (a row's word address).
__device__ __forceinline__ uint32_t row_addr_h(const uint16_t* rows, int r) {
  uint32_t a = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) a ^= ((r >> i) & 1) ? (uint32_t)rows[i] : 0u;
  return a;
}

// Address mask and LDS word vector of tile bit b of one operand (b < nbits;
// zero beyond): row bits of class row_cls use rows[idx + row_off], k bits
// 1 << hk[idx].  Branch-free: both table entries are read and the one of the
// bit's class is kept by masks.
__device__ __forceinline__ void tile_bit_h(int b, int nbits, const uint8_t* codes, const uint8_t* tab, int row_cls,
                                           int off_row, int off_k, const uint16_t* rows, int row_off, uint32_t& off,
                                           uint32_t& lds) {
  const uint32_t on = 0u - (uint32_t)(b < nbits ? 1 : 0);
  const int code = codes[b & 15];
  const int idx = code & 31;
  const uint32_t m = (uint32_t)((((code >> 5) ^ row_cls) - 1) >> 31);  // all ones for a row bit
  const uint32_t pos = ((uint32_t)tab[off_row + idx] & m) | ((uint32_t)tab[off_k + idx] & ~m);
  off = (1u << (pos & 31)) & on;
  lds = (((uint32_t)rows[(idx + row_off) & 7] & m) | ((1u << (tab[T_HK + (idx & 7)] & 31)) & ~m)) & on;
}

// Address (OR of masks) and LDS word (XOR of vectors) of tile entry e.
__device__ __forceinline__ void decode_h(uint32_t e, const uint32_t* boff, const uint32_t* blds, uint32_t& off,
                                         uint32_t& lds) {
  off = 0;
  lds = 0;
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    const uint32_t m = 0u - ((e >> b) & 1u);
    off |= boff[b] & m;
    lds ^= blds[b] & m;
  }
}

template <int P, int WM, int WN, int WK, int BM, int BN, int TK, int VA, int VB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_tile_h(StepDesc d) {
  constexpr int TM = WM * BM * 16;              // complex rows
  constexpr int TN = WN * BN * 8;               // complex columns
  constexpr int KW = TK / WK;                   // complex k per wave and k tile
  static_assert(KW % 16 == 0, "k per wave must be a multiple of 16");
  constexpr int A_WORDS = TM * TK;              // A stage: TM rows of TK words
  constexpr int STAGE = A_WORDS + 2 * TN * TK;  // + expanded B: 2 TN rows
  constexpr int SC = TN + 2;                    // float2 per LDS row of the C tile
  // VA (VB) words per global load of A (B): 4 (one 16-byte load) when the
  // two lowest tile bits are address bits 0 and 1 (the launcher checks),
  // else 1.  A thread's words of one load differ in those two bits only, so
  // their LDS words are the thread's slot XOR the uniform vectors du[u]; when
  // du = {0, 1, 2, 3} they are one aligned 16-byte LDS store.
  constexpr int A_LOADS = TM * TK / 256;
  constexpr int B_LOADS = (TK * TN + 255) / 256;
  constexpr int AV = A_LOADS / VA, BV = (B_LOADS + VB - 1) / VB;
  static_assert((VA == 1 || VA == 4) && (VB == 1 || VB == 4), "1- or 4-word loads");
  static_assert(AV * VA == A_LOADS && AV <= 16 && BV <= 16, "A loads split into whole vectors");
  constexpr int LVA = VA == 4 ? 2 : 0, LVB = VB == 4 ? 2 : 0;
  constexpr int C_ITEMS = TM * TN / 256;
  constexpr int SMEM_AB = 2 * STAGE;
  constexpr int SMEM_C = WK * TM * SC * 2;
  constexpr int SMEM = SMEM_AB > SMEM_C ? SMEM_AB : SMEM_C;
  static_assert(A_LOADS >= 1 && C_ITEMS >= 1, "tile too small");
  using VecA = typename std::conditional<VA == 4, uint4, uint32_t>::type;
  using VecB = typename std::conditional<VB == 4, uint4, uint32_t>::type;
  __shared__ __align__(16) uint32_t smem[SMEM];
  __shared__ __align__(4) uint8_t tab[TAB_BYTES];
  __shared__ uint64_t flip[2][32];
  __shared__ __align__(16) uint32_t bit_off[2][16], bit_lds[2][16];  // per tile bit of A (0) and B (1)

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = (wave / WM) % WN, wk = wave / (WM * WN);
  const uint32_t* A = reinterpret_cast<const uint32_t*>(d.A);
  const uint32_t* B = reinterpret_cast<const uint32_t*>(d.B);

  load_tables(d, tab);
  __syncthreads();
  // Padded k (fewer k bits than the stage) must read as zero in both
  // operands; other entries outside the valid tile only feed outputs that
  // are never stored.  A tile's C staging overwrites the stages, so with
  // padded k the stages are zeroed again for every tile.
  const bool pad_k = d.tk < __builtin_ctz(TK);
  const uint16_t* arow = reinterpret_cast<const uint16_t*>(tab + T_HAROW);
  const uint16_t* brow = reinterpret_cast<const uint16_t*>(tab + T_HBROW);
  const int na = d.tm + d.tk, nbt = d.tk + d.tn;
  if (tid < 32) {
    const int o = tid >> 4, b = tid & 15;
    uint32_t off, lv;
    if (o == 0) tile_bit_h(b, na, tab + T_ATILE, tab, TB_M, T_AM, T_AK, arow, 0, off, lv);
    else tile_bit_h(b, nbt, tab + T_BTILE, tab, TB_N, T_BN, T_BK, brow, 1, off, lv);
    bit_off[o][b] = off;
    bit_lds[o][b] = lv;
  }

  uint64_t baseA = 0, baseB = 0;  // tile origins in A and B (set per output tile)

  const uint64_t k_tiles = 1ull << (d.kb - d.tk);
  const uint64_t per = k_tiles >> d.ks_bits;
  const uint64_t kt0 = (uint64_t)blockIdx.y * per;
  const int khb = d.kb - d.tk;
  // Going from k tile t to t + 1 flips the logical high-k bits 0 .. ctz(t +
  // 1); flip[.][j] holds the address bits of logical bits 0 .. j.
  if (tid < khb) {
    uint64_t fa = 0, fb = 0;
    for (int i = 0; i <= tid; ++i) {
      fa |= 1ull << tab[T_AK + d.tk + i];
      fb |= 1ull << tab[T_BK + d.tk + i];
    }
    flip[0][tid] = fa;
    flip[1][tid] = fb;
  }
  __syncthreads();  // bit_off, bit_lds and flip are read from here on

  // Load slots: entry e = (tid + 256 j) * V of an operand splits into the
  // lane part tid * V (decoded once) and the uniform part 256 V j, whose
  // address mask and LDS vector combine by OR / XOR (disjoint bits).  Bits
  // at or above the operand's tile bits decode to zero, so a slot past a
  // small tile repeats a valid one (same load, same word to the same LDS
  // address): loads and stores need no bounds branches.
  uint32_t a_off_t, a_lds_t, b_off_t, b_lds_t;
  decode_h((uint32_t)tid * VA, bit_off[0], bit_lds[0], a_off_t, a_lds_t);
  decode_h((uint32_t)tid * VB, bit_off[1], bit_lds[1], b_off_t, b_lds_t);
  uint32_t ua_off[4], ua_lds[4], ub_off[4], ub_lds[4];  // tile bits 8 + log2 V + i
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ua_off[i] = __builtin_amdgcn_readfirstlane(bit_off[0][(8 + LVA + i) & 15]) * (8 + LVA + i < 16);
    ua_lds[i] = __builtin_amdgcn_readfirstlane(bit_lds[0][(8 + LVA + i) & 15]) * (8 + LVA + i < 16);
    ub_off[i] = __builtin_amdgcn_readfirstlane(bit_off[1][(8 + LVB + i) & 15]) * (8 + LVB + i < 16);
    ub_lds[i] = __builtin_amdgcn_readfirstlane(bit_lds[1][(8 + LVB + i) & 15]) * (8 + LVB + i < 16);
  }
  auto uni = [](const uint32_t* v, int j) {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) r ^= ((j >> i) & 1) ? v[i] : 0u;
    return r;
  };
  uint32_t a_du[VA], b_du[VB];  // LDS vectors of a load's words 0 .. V-1
#pragma unroll
  for (int u = 0; u < VA; ++u) a_du[u] = (u & 1 ? bit_lds[0][0] : 0u) ^ (u & 2 ? bit_lds[0][1] : 0u);
#pragma unroll
  for (int u = 0; u < VB; ++u) b_du[u] = (u & 1 ? bit_lds[1][0] : 0u) ^ (u & 2 ? bit_lds[1][1] : 0u);
  bool a_vec = false, b_vec = false;
  if constexpr (VA == 4) a_vec = a_du[1] == 1 && a_du[2] == 2 && a_du[3] == 3;
  if constexpr (VB == 4) b_vec = b_du[1] == 1 && b_du[2] == 2 && b_du[3] == 3;
  const uint32_t b_c = brow[0];

  const uint64_t ka0 = wave_scatter(kt0, tab + T_AK + d.tk, khb);
  const uint64_t kbo0 = wave_scatter(kt0, tab + T_BK + d.tk, khb);
  uint64_t ka = ka0, kbo = kbo0;
  // Two register sets of staged loads: k tile t + 2 is requested while tile
  // t is computed and tile t + 1 (requested one tile earlier) goes to the
  // other LDS stage.
  VecA ra[2][AV];
  VecB rb[2][BV];
  auto load = [&](int r) {
    const uint32_t* pa = A + (baseA + ka + a_off_t);
    const uint32_t* pb = B + (baseB + kbo + b_off_t);
#pragma unroll
    for (int j = 0; j < AV; ++j) ra[r][j] = *reinterpret_cast<const VecA*>(pa + uni(ua_off, j));
#pragma unroll
    for (int j = 0; j < BV; ++j) rb[r][j] = *reinterpret_cast<const VecB*>(pb + uni(ub_off, j));
  };
  auto swap_halves = [](uint32_t w) { return (w >> 16) | (w << 16); };
  auto store = [&](int r, int stage) {
    uint32_t* S = smem + stage * STAGE;
    uint32_t* SB = S + A_WORDS;
#pragma unroll
    for (int j = 0; j < AV; ++j) {
      const uint32_t l = a_lds_t ^ uni(ua_lds, j);
      if constexpr (VA == 4) {
        if (a_vec) {
          *reinterpret_cast<uint4*>(S + l) = ra[r][j];
        } else {
          S[l ^ a_du[0]] = ra[r][j].x;
          S[l ^ a_du[1]] = ra[r][j].y;
          S[l ^ a_du[2]] = ra[r][j].z;
          S[l ^ a_du[3]] = ra[r][j].w;
        }
      } else {
        S[l] = ra[r][j];
      }
    }
#pragma unroll
    for (int j = 0; j < BV; ++j) {
      const uint32_t l = b_lds_t ^ uni(ub_lds, j);  // row 2n; row 2n + 1 is this XOR brow[0]
      if constexpr (VB == 4) {
        const uint4 w = rb[r][j];
        if (b_vec) {
          *reinterpret_cast<uint4*>(SB + l) =
              uint4{w.x ^ 0x80000000u, w.y ^ 0x80000000u, w.z ^ 0x80000000u, w.w ^ 0x80000000u};
          *reinterpret_cast<uint4*>(SB + (l ^ b_c)) =
              uint4{swap_halves(w.x), swap_halves(w.y), swap_halves(w.z), swap_halves(w.w)};
        } else {
          const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t x = l ^ b_du[u];
            SB[x] = ws[u] ^ 0x80000000u;       // (br, -bi)
            SB[x ^ b_c] = swap_halves(ws[u]);  // (bi, br)
          }
        }
      } else {
        SB[l] = rb[r][j] ^ 0x80000000u;
        SB[l ^ b_c] = swap_halves(rb[r][j]);
      }
    }
  };
  auto advance = [&](uint64_t t) {  // load offsets from k tile kt0 + t - 1 to kt0 + t
    const int fl = __builtin_ctzll(kt0 + t);
    ka ^= flip[0][fl];
    kbo ^= flip[1][fl];
  };

  v4f acc[BM][BN];

  // Fragment word addresses: row part (lane rows 0-15 and the block rows,
  // both XORs of row vectors) and the lane's 4-word k group; each MFMA step
  // ks adds 16 words (XOR: the bits are disjoint).
  const int row = lane & 15, kg = lane >> 4;
  const uint32_t a_lane = row_addr_h(arow, row) ^ (uint32_t)(wk * KW + 4 * kg);
  const uint32_t b_lane = row_addr_h(brow, row) ^ (uint32_t)(wk * KW + 4 * kg);
  uint32_t a_frag[BM], b_frag[BN];
#pragma unroll
  for (int bm = 0; bm < BM; ++bm) a_frag[bm] = a_lane ^ row_addr_h(arow, (wm * BM + bm) * 16);
#pragma unroll
  for (int bn = 0; bn < BN; ++bn) b_frag[bn] = b_lane ^ row_addr_h(brow, (wn * BN + bn) * 16);

  // All fragment reads of a k tile are issued before its MFMAs, so the
  // MFMAs of step ks wait only for that step's reads.
  auto compute = [&](int cur) {
    const uint32_t* As = smem + cur * STAGE;
    const uint32_t* Bs = As + A_WORDS;
    uint4 av[KW / 16][BM], bv[KW / 16][BN];
#pragma unroll
    for (int ks = 0; ks < KW / 16; ++ks) {
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
        av[ks][bm] = *reinterpret_cast<const uint4*>(As + (a_frag[bm] ^ (uint32_t)(16 * ks)));
#pragma unroll
      for (int bn = 0; bn < BN; ++bn)
        bv[ks][bn] = *reinterpret_cast<const uint4*>(Bs + (b_frag[bn] ^ (uint32_t)(16 * ks)));
    }
#pragma unroll
    for (int ks = 0; ks < KW / 16; ++ks)
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn) {
          if constexpr (P == 1)
            acc[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                __builtin_bit_cast(v8h, av[ks][bm]), __builtin_bit_cast(v8h, bv[ks][bn]), acc[bm][bn], 0, 0, 0);
          else
            acc[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(v8bf, av[ks][bm]), __builtin_bit_cast(v8bf, bv[ks][bn]), acc[bm][bn], 0, 0, 0);
        }
  };
  // One k tile: stage it & 1 holds tile it, register set x holds tile it + 1.
  auto step = [&](uint64_t it, int x) {
    if (it + 2 < per) {
      advance(it + 2);
      load(x ^ 1);
    }
    compute((int)(it & 1));
    if (it + 1 < per) store(x, (int)(it & 1) ^ 1);
    __syncthreads();
  };

  // Output tiles are dealt grid-stride (the launch holds about as many
  // workgroups as are resident), so the set-up above is paid once per
  // workgroup and a tile's stores drain while the next tile loads.
  const uint64_t n_mt = 1ull << (d.mb - d.tm), n_nt = 1ull << (d.nb - d.tn);
  const uint64_t batch = blockIdx.z;
  for (uint64_t tx = blockIdx.x; tx < n_mt * n_nt; tx += gridDim.x) {
    uint64_t mt, nt;
    tile_of(tx, n_mt, n_nt, mt, nt);
    baseA = wave_scatter(mt, tab + T_AM + d.tm, d.mb - d.tm) + wave_scatter(batch, tab + T_AB, d.bb);
    baseB = wave_scatter(nt, tab + T_BN + d.tn, d.nb - d.tn) + wave_scatter(batch, tab + T_BB, d.bb);
    ka = ka0;
    kbo = kbo0;
    if (pad_k) {
      for (int i = tid; i < SMEM_AB; i += 256) smem[i] = 0u;
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    load(0);
    if (per > 1) {
      advance(1);
      load(1);
    }
    store(0, 0);
    __syncthreads();
    for (uint64_t it = 0; it < per; it += 2) {
      step(it, 1);
      if (it + 1 < per) step(it + 1, 0);
    }
    // Accumulators -> LDS tile (rows m, interleaved re/im columns).
    float* Cf = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = (wm * BM + bm) * 16 + 4 * kg + i;
          const int col = (wn * BN + bn) * 16 + row;  // 2n + part
          Cf[(wk * TM + m) * (2 * SC) + col] = acc[bm][bn][i];
        }
    __syncthreads();
    store_c_tile<P, TM, WK, SC, C_ITEMS>(d, tab, reinterpret_cast<const float2*>(smem), mt, nt, batch);
    __syncthreads();  // the next tile's staging overwrites the C tile
  }
}

// Deterministic FP64 sum of split-K partials (blocked summation, Sec. V-B /
// Eq. 3: each FP32 chain covers only K / splits terms).  A workgroup takes
// 256 / 2^rb consecutive output entries and 2^rb split rows (rb <= 4): thread
// (row r, column c) sums splits r, r + 2^rb, ... of entry c in FP64, then row
// 0 adds the row sums in row order, so the result does not depend on timing.
// Loads of one row are consecutive entries (coalesced); the 2^rb rows keep
// that many independent load streams per entry in flight.
template <int P>
__global__ __launch_bounds__(256) void k_reduce(StepDesc d, int rb) {
  __shared__ double2 red[256];
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  const float2* part = reinterpret_cast<const float2*>(d.part);
  const uint64_t splits = 1ull << d.ks_bits;
  const int cols = 256 >> rb;
  const int r = threadIdx.x / cols, cl = threadIdx.x % cols;
  float mx = 0.f;
  for (uint64_t c0 = (uint64_t)blockIdx.x * cols; c0 < c_elems; c0 += (uint64_t)gridDim.x * cols) {
    const uint64_t c = c0 + cl;
    double sx = 0, sy = 0;
    if (c < c_elems) {
      uint64_t sp = r;
      for (; sp + 3 * (1ull << rb) < splits; sp += 4ull << rb) {
        float2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = part[(sp + ((uint64_t)u << rb)) * c_elems + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          sx += v[u].x;
          sy += v[u].y;
        }
      }
      for (; sp < splits; sp += 1ull << rb) {
        const float2 v = part[sp * c_elems + c];
        sx += v.x;
        sy += v.y;
      }
    }
    red[threadIdx.x] = make_double2(sx, sy);
    __syncthreads();
    if (r == 0 && c < c_elems) {
      for (int q = 1; q < (1 << rb); ++q) {
        sx += red[q * cols + cl].x;
        sy += red[q * cols + cl].y;
      }
      if (d.mode == EPI_ACC64) {
        double2* acc = reinterpret_cast<double2*>(d.acc);
        double2 o = acc[c];
        o.x += sx * d.acc_scale;
        o.y += sy * d.acc_scale;
        acc[c] = o;
      } else if constexpr (P == 0) {
        const float2 v = make_float2((float)sx, (float)sy);
        reinterpret_cast<float2*>(d.C)[c] = v;
        mx = fmaxf(mx, absmax2(v));
      } else {
        const float2 v = make_float2((float)(sx * d.out_scale), (float)(sy * d.out_scale));
        reinterpret_cast<uint32_t*>(d.C)[c] = pack<P>(v);
        mx = fmaxf(mx, absmax2(v));
      }
    }
    __syncthreads();
  }
  record_max(d, mx);
}

// ---------------------------------------------------------------- reverse pass
__global__ __launch_bounds__(256) void k_seed(const double2* w, float2* adj, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) adj[i] = make_float2((float)w[i].x, (float)w[i].y);
}

// One thread per single-qubit gate leaf: its adjoint (at most 4 entries) is
// added into the gate's 4 gradient entries at the positions its sliced
// indices take in this slice.
__global__ __launch_bounds__(256) void k_grad(const GradEntry* tab, int n_entries, const char* ws, uint64_t slice,
                                              double2* grad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_entries) return;
  const GradEntry e = tab[i];
  const float2* adj = reinterpret_cast<const float2*>(ws + e.adj_offset);
  uint32_t base = 0;
  for (int j = 0; j < e.n_sliced; ++j) base |= (uint32_t)((slice >> e.slice_bit[j]) & 1ull) << e.slice_pos[j];
  for (int r = 0; r < (1 << e.rank); ++r) {
    uint32_t full = base;
    for (int b = 0; b < e.rank; ++b) full |= (uint32_t)((r >> b) & 1) << e.full_pos[b];
    const float2 v = adj[r];
    double2 o = grad[4 * e.gate + full];
    o.x += v.x;
    o.y += v.y;
    grad[4 * e.gate + full] = o;
  }
}

// acc[i] += src[i] (complex128): adds a verified partial sum of slices into
// the caller's result.
__global__ __launch_bounds__(256) void k_accumulate(double2* acc, const double2* src, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    double2 o = acc[i];
    const double2 v = src[i];
    o.x += v.x;
    o.y += v.y;
    acc[i] = o;
  }
}

hipError_t launch_accumulate(double* acc, const double* src, uint64_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_accumulate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<double2*>(acc), reinterpret_cast<const double2*>(src), n);
  return hipGetLastError();
}

hipError_t launch_seed(const double* w, float* adj, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_seed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(w), reinterpret_cast<float2*>(adj), n);
  return hipGetLastError();
}

hipError_t launch_grad(const GradEntry* tab, int n_entries, const char* ws, uint64_t slice, double* grad,
                       hipStream_t s) {
  if (n_entries == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad, dim3((unsigned)((n_entries + 255) / 256)), dim3(256), 0, s, tab, n_entries, ws, slice,
                     reinterpret_cast<double2*>(grad));
  return hipGetLastError();
}

// ---------------------------------------------------------------- launch
// Launch with optional timing: with an event pair the launch goes through
// hipExtLaunchKernelGGL, whose events carry the kernel's own start and end
// (no dispatch gap inside the measured interval).
struct Timing {
  hipEvent_t e0 = nullptr, e1 = nullptr;
};
template <typename F, typename... Args>
static void launch_k(F kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, Timing t, Args... args) {
  if (t.e0) hipExtLaunchKernelGGL(kernel, grid, block, lds, s, t.e0, t.e1, 0, args...);
  else hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

template <int P>
static hipError_t launch_stem(const StepDesc& d, dim3 grid, hipStream_t s, Timing t) {
#define MITNC_STEM(KB, NB)                                                \
  if (d.kb == KB && d.nb == NB) {                                         \
    launch_k(k_stem<P, KB, NB>, grid, dim3(256), 0, s, t, d);             \
    return hipGetLastError();                                             \
  }
  MITNC_STEM(0, 0) MITNC_STEM(0, 1) MITNC_STEM(0, 2)
  MITNC_STEM(1, 0) MITNC_STEM(1, 1) MITNC_STEM(1, 2)
  MITNC_STEM(2, 0) MITNC_STEM(2, 1) MITNC_STEM(2, 2)
  MITNC_STEM(3, 0) MITNC_STEM(3, 1) MITNC_STEM(3, 2)
  MITNC_STEM(4, 0) MITNC_STEM(4, 1) MITNC_STEM(4, 2)
#undef MITNC_STEM
  return hipErrorInvalidValue;
}

// Stream steps.  Each wave takes iters iterations of R row blocks.  The
// grid holds as many waves as the device keeps resident at once for the
// kernel (its occupancy times the SIMDs, rounded down to a power of two, at
// most 2^MaxLog), so no wave waits for a second round; fewer when the step
// has fewer row-block groups.  Measured on the benchmark workload: 8192 waves
// for complex64 (2498 -> 2513 slices/s against 4096), 4096 for the 16-bit
// kernels (8192 slowed them by 6 %).
template <auto Kern, int MaxLog>
static int stream_wave_cap_log() {
  static int cap = -1;  // per kernel; devices of one process are alike
  if (cap < 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, Kern, 256, 0) != hipSuccess || per_cu < 1 || cus < 1)
      return 12;
    const long waves = (long)per_cu * 4 * cus;
    int l = 0;
    while (l < MaxLog && (2L << l) <= waves) ++l;
    cap = l;
  }
  return cap;
}

template <auto Kern, int MaxLog>
static hipError_t launch_stream_k(const StepDesc& d, int rl, int cs, hipStream_t s, Timing t) {
  const int ngl = d.mb - 4 + d.bb - rl;  // log2 of row-block groups of all batch indices
  const int cap = stream_wave_cap_log<Kern, MaxLog>();
  const int wl = ngl < cap ? ngl : cap;        // log2 waves (>= 0 since mb >= 8)
  if (wl < d.bb) return hipErrorInvalidValue;  // a wave must stay inside one batch index
  const uint32_t iters = 1u << (ngl - wl);
  // fewer than 4 waves: one workgroup, idle waves exit; 2^cs column groups
  const dim3 grid(wl >= 2 ? 1u << (wl - 2) : 1u, 1u << cs);
  launch_k(Kern, grid, dim3(256), 0, s, t, d, iters);
  return hipGetLastError();
}

// Column groups of a stream launch with few waves: a step with few rows
// would leave most of the chip idle while each wave stores all N columns,
// so up to 2^10 waves the column blocks are dealt to 2^cs launch columns
// (each re-reads its rows of A; kept to K 2^cs <= N so that the extra reads
// stay below the output's bytes).
static int stream_column_split(const StepDesc& d, int rl, int nbl, int cap) {
  const int ngl = d.mb - 4 + d.bb - rl;
  const int wl = ngl < cap ? ngl : cap;
  int cs = wl < 10 ? (10 - wl < nbl ? 10 - wl : nbl) : 0;
  while (cs > 0 && d.kb + cs > d.nb) --cs;
  return cs;
}

// 16-bit storage: KS8 = 2^ksl k steps of 8, NB8 = 2^nbl column blocks of 8.
template <int P>
static hipError_t launch_stream_h(const StepDesc& d, hipStream_t s, Timing t) {
  const int ksl = d.kb > 3 ? d.kb - 3 : 0, nbl = d.nb > 3 ? d.nb - 3 : 0;
  if (!stream_fits(d.mb, d.nb, d.kb, d.bb) || ksl + nbl > 4) return hipErrorInvalidValue;
  if (!stream_rows_sorted(d) || !stream_offsets_fit(d, 4, d.mode == EPI_ACC64 ? 16 : 4)) return hipErrorInvalidValue;
  const int rl = kStreamRowsH > ksl ? kStreamRowsH - ksl : 0;  // log2 R, as in the kernel
  const int cs = stream_column_split(d, rl, nbl, 12);
  const int nbg = nbl - cs;  // column blocks per launch column
#define MITNC_STREAMH(KSL, NBL) \
  if (ksl == KSL && nbg == NBL) return launch_stream_k<k_stream_h<P, 1 << KSL, 1 << NBL>, 12>(d, rl, cs, s, t);
  MITNC_STREAMH(0, 0) MITNC_STREAMH(0, 1) MITNC_STREAMH(0, 2) MITNC_STREAMH(0, 3)
  MITNC_STREAMH(1, 0) MITNC_STREAMH(1, 1) MITNC_STREAMH(1, 2) MITNC_STREAMH(1, 3)
  MITNC_STREAMH(2, 0) MITNC_STREAMH(2, 1) MITNC_STREAMH(2, 2)
  MITNC_STREAMH(3, 0) MITNC_STREAMH(3, 1)
#undef MITNC_STREAMH
  return hipErrorInvalidValue;
}

// complex64: KS = 2^ksl k steps of 4, NBLK = 2^nbl column blocks of 16.
static hipError_t launch_stream_f(const StepDesc& d, hipStream_t s, Timing t) {
  constexpr int P = 0;
  const int ksl = d.kb > 2 ? d.kb - 2 : 0, nbl = d.nb > 4 ? d.nb - 4 : 0;
  if (!stream_fits(d.mb, d.nb, d.kb, d.bb)) return hipErrorInvalidValue;
  if (!stream_rows_sorted(d) || !stream_offsets_fit(d, 8, d.mode == EPI_ACC64 ? 16 : 8)) return hipErrorInvalidValue;
  const int rl = kStreamRowsF > ksl ? kStreamRowsF - ksl : 0;  // log2 R, as in the kernel
  const int cs = stream_column_split(d, rl, nbl, 13);
  const int nbg = nbl - cs;  // column blocks per launch column
#define MITNC_STREAM(KSL, NBL) \
  if (ksl == KSL && nbg == NBL) return launch_stream_k<k_stream<P, 1 << KSL, 1 << NBL>, 13>(d, rl, cs, s, t);
  MITNC_STREAM(0, 0) MITNC_STREAM(1, 0) MITNC_STREAM(2, 0) MITNC_STREAM(3, 0) MITNC_STREAM(4, 0)
  MITNC_STREAM(0, 1) MITNC_STREAM(1, 1) MITNC_STREAM(2, 1) MITNC_STREAM(3, 1)
  MITNC_STREAM(0, 2) MITNC_STREAM(1, 2) MITNC_STREAM(2, 2)
#undef MITNC_STREAM
  return hipErrorInvalidValue;
}

template <int P>
static hipError_t launch_stream(const StepDesc& d, hipStream_t s, Timing t) {
  if constexpr (P == 0) return launch_stream_f(d, s, t);
  else return launch_stream_h<P>(d, s, t);
}

// Skinny split-K: one 64-lane workgroup per (k split, batch index).
static hipError_t launch_skinny(const StepDesc& d, hipStream_t s, Timing t) {
  if (!skinny_fits(d.mb, d.nb, d.kb, d.bb, d.ks_bits)) return hipErrorInvalidValue;
  const dim3 grid(1u << d.ks_bits, 1u << d.bb);
#define MITNC_SKINNY(MB, NB)                                          \
  if (d.mb == MB && d.nb == NB) {                                     \
    launch_k(k_skinny<MB, NB>, grid, dim3(64), 0, s, t, d);           \
    return hipGetLastError();                                         \
  }
  MITNC_SKINNY(0, 0) MITNC_SKINNY(0, 1) MITNC_SKINNY(0, 2) MITNC_SKINNY(0, 3) MITNC_SKINNY(0, 4)
  MITNC_SKINNY(1, 0) MITNC_SKINNY(1, 1) MITNC_SKINNY(1, 2) MITNC_SKINNY(1, 3)
  MITNC_SKINNY(2, 0) MITNC_SKINNY(2, 1) MITNC_SKINNY(2, 2)
  MITNC_SKINNY(3, 0) MITNC_SKINNY(3, 1)
  MITNC_SKINNY(4, 0)
#undef MITNC_SKINNY
  return hipErrorInvalidValue;
}

// Address bit of tile bit `code` in A (is_a) or B.
static int tile_bit_pos(const StepDesc& d, uint8_t code, bool is_a) {
  const int cls = code >> 5, idx = code & 31;
  if (is_a) return cls == TB_M ? d.am[idx] : d.ak[idx];
  return cls == TB_K ? d.bk[idx] : d.bn[idx];
}

// 16-byte loads of A (B) apply when the plan chose them (StepDesc::vec_a,
// vec_b), the two lowest tile bits are the operand's address bits 0 and 1
// (four consecutive words of a tile are then consecutive in memory) and the
// operand is 16-byte aligned.
static bool tile_vec_a(const StepDesc& d) {
  return d.vec_a == 4 && d.tm + d.tk >= 2 && tile_bit_pos(d, d.a_tile[0], true) == 0 &&
         tile_bit_pos(d, d.a_tile[1], true) == 1 && (reinterpret_cast<uintptr_t>(d.A) & 15) == 0;
}
static bool tile_vec_b(const StepDesc& d) {
  return d.vec_b == 4 && d.tk + d.tn >= 2 && tile_bit_pos(d, d.b_tile[0], false) == 0 &&
         tile_bit_pos(d, d.b_tile[1], false) == 1 && (reinterpret_cast<uintptr_t>(d.B) & 15) == 0;
}

template <int P, int WM, int WN, int WK, int BM, int BN, int TK>
static void launch_tile_h(const StepDesc& d, dim3 grid, hipStream_t s, Timing t) {
  const bool va = tile_vec_a(d), vb = tile_vec_b(d);
  if (va && vb) launch_k(k_tile_h<P, WM, WN, WK, BM, BN, TK, 4, 4>, grid, dim3(256), 0, s, t, d);
  else if (va) launch_k(k_tile_h<P, WM, WN, WK, BM, BN, TK, 4, 1>, grid, dim3(256), 0, s, t, d);
  else if (vb) launch_k(k_tile_h<P, WM, WN, WK, BM, BN, TK, 1, 4>, grid, dim3(256), 0, s, t, d);
  else launch_k(k_tile_h<P, WM, WN, WK, BM, BN, TK, 1, 1>, grid, dim3(256), 0, s, t, d);
}

#ifndef MITNC_TALL_SLOTS_PER_CU
#define MITNC_TALL_SLOTS_PER_CU 2ull
#endif

template <int P>
static hipError_t launch_p(int kclass, StepDesc d, hipStream_t s, Timing t) {
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  hipError_t e = hipSuccess;
  switch (kclass) {
    case MITNC_K_SMALL: {
      dim3 grid((unsigned)((c_elems + 255) / 256));
      if (small_bounded(d.mb, d.nb, d.kb, d.bb)) launch_k(k_small<P, true>, grid, dim3(256), 0, s, t, d);
      else launch_k(k_small<P, false>, grid, dim3(256), 0, s, t, d);
      e = hipGetLastError();
      break;
    }
    case MITNC_K_STEM: {
      const int lowb = d.mb < 8 ? d.mb : 8;
      const uint64_t n_mhi = 1ull << (d.mb - lowb);
      dim3 grid((unsigned)(n_mhi < 16384 ? n_mhi : 16384), (unsigned)(1ull << d.bb));
      e = launch_stem<P>(d, grid, s, t);
      break;
    }
    case MITNC_K_STREAM:
      e = launch_stream<P>(d, s, t);
      break;
    case MITNC_K_TILE:
    case MITNC_K_TALL:
    case MITNC_K_SPLITK: {
      // The descriptor's tile bits must fit the tile the kernel was compiled
      // for (LDS slots are sized from it).
      const TileGeom g = P == 0 ? (kclass == MITNC_K_TILE ? geom_tile() : kclass == MITNC_K_TALL ? geom_tall() : geom_splitk())
                                : (kclass == MITNC_K_TILE ? geom_tile_h()
                                   : kclass == MITNC_K_TALL ? geom_tall_h() : geom_splitk_h());
      if (d.tm > g.tm_bits || d.tn > g.tn_bits || d.tk > g.tk_bits || d.tm < 0 || d.tn < 0 || d.tk < 0 ||
          d.ks_bits > d.kb - d.tk)
        return hipErrorInvalidValue;
      const int final_mode = d.mode;
      if (d.ks_bits > 0) d.mode = EPI_PARTIAL;
      // Output tiles per split and batch index are dealt grid-stride by the
      // kernels: the launch holds about the resident workgroup count (2 per
      // CU), in multiples of 8 (one per XCD), or every tile when there are
      // fewer.
      const uint64_t n_tiles = 1ull << ((d.mb - d.tm) + (d.nb - d.tn));
      const uint64_t yz = (1ull << d.ks_bits) << d.bb;
      const uint64_t slots = (kclass == MITNC_K_TALL ? MITNC_TALL_SLOTS_PER_CU : 2ull) * 256;
      const uint64_t cap = yz * 8 >= slots ? 8 : (slots / yz) & ~7ull;
      dim3 grid((unsigned)(n_tiles < cap ? n_tiles : cap), (unsigned)(1ull << d.ks_bits), (unsigned)(1ull << d.bb));
      if constexpr (P == 0) {
        if (kclass == MITNC_K_TILE)
          launch_k(k_tile<MITNC_TILE_WM, MITNC_TILE_WN, MITNC_TILE_WK, MITNC_TILE_BM, MITNC_TILE_BN, MITNC_TILE_TK>,
                   grid, dim3(256), 0, s, t, d);
        else if (kclass == MITNC_K_TALL)
          launch_k(k_tile<4, 1, 1, 2, 1, 16>, grid, dim3(256), 0, s, t, d);
        else if (skinny_fits(d.mb, d.nb, d.kb, d.bb, d.ks_bits))
          e = launch_skinny(d, s, t);
        else
          launch_k(k_tile<1, 1, 4, 1, 1, 64>, grid, dim3(256), 0, s, t, d);
      } else {
        if (kclass == MITNC_K_TILE)
          launch_tile_h<P, MITNC_TILEH_WM, MITNC_TILEH_WN, MITNC_TILEH_WK, MITNC_TILEH_BM, MITNC_TILEH_BN,
                        MITNC_TILEH_TK>(d, grid, s, t);
        else if (kclass == MITNC_K_TALL)
          launch_tile_h<P, 4, 1, 1, 2, 2, 32>(d, grid, s, t);
        else
          launch_tile_h<P, 1, 1, 4, 1, 2, 128>(d, grid, s, t);
      }
      if (e == hipSuccess) e = hipGetLastError();
      if (e != hipSuccess || d.ks_bits == 0) return e;
      d.mode = final_mode;
      // split rows per workgroup: up to 16, fewer when the splits are few
      const int rb = d.ks_bits < 4 ? d.ks_bits : 4;
      const uint64_t groups = (c_elems + (256 >> rb) - 1) / (256 >> rb);
      hipLaunchKernelGGL((k_reduce<P>), dim3((unsigned)(groups < 8192 ? groups : 8192)), dim3(256), 0, s, d, rb);
      return hipGetLastError();
    }
    default:
      return hipErrorInvalidValue;
  }
  return e;
}

template <int P>
static hipError_t launch_section_p(const SectionDesc& sd, unsigned grid, size_t lds, hipStream_t s, Timing t) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_section<P>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSectionMaxLds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  launch_k(k_section<P>, dim3(grid), dim3(256), (uint32_t)lds, s, t, sd);
  return hipGetLastError();
}

hipError_t launch_section(const SectionDesc& sd, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  // Host checks of what the kernel assumes: tile sizes, step count, LDS.
  if (sd.n_steps < 1 || sd.n_steps > kMaxSectionSteps || sd.t_in < 8 || sd.t_out < 8 || sd.t_in > 12 ||
      sd.t_out > 12 ||
      sd.t_in > kMaxTileBits || sd.t_out > kMaxTileBits || (1 << sd.t_in) > sd.tile_max ||
      (1 << sd.t_out) > sd.tile_max || sd.tile_max > (1 << kMaxTileBits) || sd.outer_bits < 0 ||
      sd.outer_bits > 32)
    return hipErrorInvalidValue;
  for (int j = 0; j < sd.n_steps; ++j) {
    const TileStep& t = sd.st[j];
    if (t.mb < 4 || t.mb + t.kb > kMaxTileBits || t.mb + t.nb > kMaxTileBits || t.kb > 6 || t.nb > 6 ||
        (t.kb > 2 ? t.kb - 2 : 0) + (t.nb > 4 ? t.nb - 4 : 0) > 4 ||
        (1 << (t.mb + t.kb)) > sd.tile_max || (1 << (t.mb + t.nb)) > sd.tile_max)
      return hipErrorInvalidValue;
  }
  if (sd.tb_bits < 0 || sd.tb_bits > sd.outer_bits || sd.stride_bits < sd.t_in || sd.stride_bits < sd.t_out ||
      sd.stride_bits + sd.tb_bits > 12 || (1 << (sd.stride_bits + sd.tb_bits)) > sd.tile_max)
    return hipErrorInvalidValue;
  for (int j = 0; j < sd.n_steps; ++j) {
    const TileStep& t = sd.st[j];
    if (t.mb + t.kb > sd.stride_bits || t.mb + t.nb > sd.stride_bits) return hipErrorInvalidValue;
  }
  const size_t lds = (2ull * sd.tile_max + sd.b_total) * sizeof(float2);
  if (lds > kSectionMaxLds) return hipErrorInvalidValue;
  const uint64_t tiles = 1ull << (sd.outer_bits - sd.tb_bits);
  const unsigned per_cu = lds > kSectionMaxLds / 2 ? 1 : 2;
  const unsigned grid = (unsigned)(tiles < 256ull * per_cu ? tiles : 256ull * per_cu);
  const Timing t{ev0, ev1};
  switch (sd.prec) {
    case MITNC_C64: return launch_section_p<0>(sd, grid, lds, s, t);
    case MITNC_CF16: return launch_section_p<1>(sd, grid, lds, s, t);
    case MITNC_CBF16: return launch_section_p<2>(sd, grid, lds, s, t);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step(int kclass, const StepDesc& d, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const Timing t{ev0, ev1};
  switch (d.prec) {
    case MITNC_C64: return launch_p<0>(kclass, d, s, t);
    case MITNC_CF16: return launch_p<1>(kclass, d, s, t);
    case MITNC_CBF16: return launch_p<2>(kclass, d, s, t);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mitnc
