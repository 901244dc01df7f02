// Contraction kernels for gfx950 (CDNA4).
//
// Every kernel computes one pairwise contraction described by a StepDesc:
//   C[b, m, n] = sum_k A[b, m, k] * B[b, k, n]     (complex)
// with each logical bit scattered to an arbitrary address bit of each operand
// (TTGT of Sec. II-A with the transposes fused into the loads, Sec. V-A).
//
// Complex GEMM on MFMA (4M form): with A viewed as a real M x 2K matrix
// A'[m][2k + p] = (Re, Im)[p] of A[m][k] and B expanded into 2 x 2 real blocks
// B'[2k .. 2k+1][2n .. 2n+1] = [[br, bi], [-bi, br]], the real product A' B'
// holds Re C in even and Im C in odd columns (8 M K N real flops, the complex
// flop count).  One v_mfma_f32_16x16x4_f32 covers 16 rows, 8 complex columns
// and 2 complex k.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace mitnc {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t scatter_bits(uint64_t x, const uint8_t* pos, int n) {
  uint64_t r = 0;
  for (int i = 0; i < n; ++i) r |= ((x >> i) & 1ull) << pos[i];
  return r;
}

__device__ __forceinline__ uint64_t gather_bits(uint64_t a, const uint8_t* pos, int n) {
  uint64_t r = 0;
  for (int i = 0; i < n; ++i) r |= ((a >> pos[i]) & 1ull) << i;
  return r;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ void epilogue_store(const StepDesc& d, uint64_t addr, float2 v, uint64_t split,
                                               uint64_t c_elems) {
  if (d.mode == EPI_STORE) {
    reinterpret_cast<float2*>(d.C)[addr] = v;
  } else if (d.mode == EPI_ACC64) {
    double2* acc = reinterpret_cast<double2*>(d.acc);
    double2 o = acc[addr];
    o.x += (double)v.x;
    o.y += (double)v.y;
    acc[addr] = o;
  } else {
    reinterpret_cast<float2*>(d.part)[split * c_elems + addr] = v;
  }
}

// ---------------------------------------------------------------- small steps
// One thread per output entry, direct loads; correct for any shape.
__global__ __launch_bounds__(256) void k_small(StepDesc d) {
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  const uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= c_elems) return;
  const float2* A = reinterpret_cast<const float2*>(d.A);
  const float2* B = reinterpret_cast<const float2*>(d.B);
  uint64_t m = gather_bits(c, d.cm, d.mb), n = gather_bits(c, d.cn, d.nb), b = gather_bits(c, d.cb, d.bb);
  uint64_t ao = scatter_bits(m, d.am, d.mb) + scatter_bits(b, d.ab, d.bb);
  uint64_t bo = scatter_bits(n, d.bn, d.nb) + scatter_bits(b, d.bbt, d.bb);
  const uint64_t K = 1ull << d.kb;
  float2 s = make_float2(0.f, 0.f);
  for (uint64_t k = 0; k < K; ++k) {
    float2 a = A[ao + scatter_bits(k, d.ak, d.kb)];
    float2 bv = B[bo + scatter_bits(k, d.bk, d.kb)];
    s.x += a.x * bv.x - a.y * bv.y;
    s.y += a.x * bv.y + a.y * bv.x;
  }
  epilogue_store(d, c, s, 0, c_elems);
}

// ---------------------------------------------------------------- stem steps
// A big tensor absorbs a small matrix (K <= 16, N <= 4): one thread per row m
// (and batch index), the small matrix in LDS.  Consecutive threads take
// consecutive m, whose bits are A's lowest non-contracted address bits, so
// loads and stores are coalesced whatever the bit positions of k and n.
template <int KB, int NB>
__global__ __launch_bounds__(256) void k_stem(StepDesc d) {
  constexpr int K = 1 << KB, N = 1 << NB;
  __shared__ float2 Bs[K * N];
  __shared__ uint32_t ka[K], nc[N];
  const uint64_t batch = blockIdx.y;
  const int t = threadIdx.x;
  const float2* A = reinterpret_cast<const float2*>(d.A);
  const float2* B = reinterpret_cast<const float2*>(d.B);
  const uint64_t bB = scatter_bits(batch, d.bbt, d.bb);
  if (t < K * N) {
    int k = t / N, n = t % N;
    Bs[t] = B[bB + scatter_bits(k, d.bk, KB) + scatter_bits(n, d.bn, NB)];
  }
  if (t < K) ka[t] = (uint32_t)scatter_bits(t, d.ak, KB);
  if (t < N) nc[t] = (uint32_t)scatter_bits(t, d.cn, NB);
  __syncthreads();
  const int lowb = d.mb < 8 ? d.mb : 8;
  if (t >= (1 << lowb)) return;
  const uint64_t mhi = blockIdx.x;  // high m bits (uniform)
  uint64_t aoff = scatter_bits(mhi, d.am + lowb, d.mb - lowb) + scatter_bits(batch, d.ab, d.bb);
  uint64_t coff = scatter_bits(mhi, d.cm + lowb, d.mb - lowb) + scatter_bits(batch, d.cb, d.bb);
  aoff += scatter_bits(t, d.am, lowb);
  coff += scatter_bits(t, d.cm, lowb);
  float2 a[K];
#pragma unroll
  for (int k = 0; k < K; ++k) a[k] = A[aoff + ka[k]];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    float2 s = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float2 b = Bs[k * N + n];
      s.x += a[k].x * b.x - a[k].y * b.y;
      s.y += a[k].x * b.y + a[k].y * b.x;
    }
    epilogue_store(d, coff + nc[n], s, 0, 1ull << (d.mb + d.nb + d.bb));
  }
}

// ---------------------------------------------------------------- MFMA tiles
// Workgroup of 4 waves computes a TM x TN complex tile of C over a range of
// TK-wide k tiles.  WM x WN x WK waves: WM x WN split the tile, WK split each
// k tile (their partial tiles are summed in LDS in a fixed order).
// Global -> LDS: each thread owns fixed tile elements enumerated in the
// operand's address order (coalesced), and writes them to the LDS position of
// their logical (m, k) / (k, n) coordinate: the permutation happens here.
template <int WM, int WN, int WK, int BM, int BN, int TK>
__global__ __launch_bounds__(256) void k_tile(StepDesc d) {
  constexpr int TM = WM * BM * 16;
  constexpr int TN = WN * BN * 8;
  constexpr int SA = TM + (TM >= 64 ? 16 : 0);  // floats per LDS row of A (row = 2k + part)
  constexpr int SB = TN + (TN >= 32 ? 8 : 0);   // float2 per LDS row of B (row = k)
  constexpr int SC = 2 * TN + 2;                // floats per LDS row of the C tile
  constexpr int A_LOADS = TM * TK / 256;
  constexpr int B_LOADS = (TK * TN + 255) / 256;
  constexpr int C_ITEMS = TM * TN / 256;
  constexpr int SMEM_AB = 2 * TK * SA + 2 * TK * SB;
  constexpr int SMEM_C = WK * TM * SC;
  constexpr int SMEM = SMEM_AB > SMEM_C ? SMEM_AB : SMEM_C;
  static_assert(A_LOADS >= 1 && C_ITEMS >= 1, "tile too small");
  __shared__ float smem[SMEM];
  float* As = smem;
  float2* Bs = reinterpret_cast<float2*>(smem + 2 * TK * SA);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = (wave / WM) % WN, wk = wave / (WM * WN);
  const float2* A = reinterpret_cast<const float2*>(d.A);
  const float2* B = reinterpret_cast<const float2*>(d.B);

  const uint64_t n_mt = 1ull << (d.mb - d.tm);
  const uint64_t mt = blockIdx.x % n_mt, nt = blockIdx.x / n_mt;
  const uint64_t batch = blockIdx.z;
  const uint64_t baseA = scatter_bits(mt, d.am + d.tm, d.mb - d.tm) + scatter_bits(batch, d.ab, d.bb);
  const uint64_t baseB = scatter_bits(nt, d.bn + d.tn, d.nb - d.tn) + scatter_bits(batch, d.bbt, d.bb);

  // Per-thread load slots.
  uint32_t a_off[A_LOADS];
  int a_lds[A_LOADS];
  const int na = d.tm + d.tk;
#pragma unroll
  for (int j = 0; j < A_LOADS; ++j) {
    int e = tid + 256 * j;
    a_lds[j] = -1;
    a_off[j] = 0;
    if (e < (1 << na)) {
      uint32_t off = 0;
      int mi = 0, ki = 0;
      for (int b = 0; b < na; ++b) {
        int bit = (e >> b) & 1;
        uint8_t code = d.a_tile[b];
        int idx = code & 31;
        if ((code >> 5) == TB_M) {
          mi |= bit << idx;
          off |= (uint32_t)bit << d.am[idx];
        } else {
          ki |= bit << idx;
          off |= (uint32_t)bit << d.ak[idx];
        }
      }
      a_off[j] = off;
      a_lds[j] = 2 * ki * SA + mi;
    }
  }
  uint32_t b_off[B_LOADS];
  int b_lds[B_LOADS];
  const int nbt = d.tk + d.tn;
#pragma unroll
  for (int j = 0; j < B_LOADS; ++j) {
    int e = tid + 256 * j;
    b_lds[j] = -1;
    b_off[j] = 0;
    if (e < (1 << nbt)) {
      uint32_t off = 0;
      int ni = 0, ki = 0;
      for (int b = 0; b < nbt; ++b) {
        int bit = (e >> b) & 1;
        uint8_t code = d.b_tile[b];
        int idx = code & 31;
        if ((code >> 5) == TB_N) {
          ni |= bit << idx;
          off |= (uint32_t)bit << d.bn[idx];
        } else {
          ki |= bit << idx;
          off |= (uint32_t)bit << d.bk[idx];
        }
      }
      b_off[j] = off;
      b_lds[j] = ki * SB + ni;
    }
  }
  // Zero the LDS tiles once: entries outside the valid tile stay zero, so
  // padded k never contributes and padded rows/columns only feed outputs that
  // are never stored.
  for (int i = tid; i < SMEM_AB; i += 256) smem[i] = 0.f;

  const uint64_t k_tiles = 1ull << (d.kb - d.tk);
  const uint64_t per = k_tiles >> d.ks_bits;
  const uint64_t kt0 = (uint64_t)blockIdx.y * per, kt1 = kt0 + per;
  const int khb = d.kb - d.tk;

  float2 ra[A_LOADS], rb[B_LOADS];
  auto load = [&](uint64_t kt) {
    uint64_t ka = scatter_bits(kt, d.ak + d.tk, khb);
    uint64_t kbo = scatter_bits(kt, d.bk + d.tk, khb);
#pragma unroll
    for (int j = 0; j < A_LOADS; ++j) ra[j] = a_lds[j] >= 0 ? A[baseA + ka + a_off[j]] : make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < B_LOADS; ++j) rb[j] = b_lds[j] >= 0 ? B[baseB + kbo + b_off[j]] : make_float2(0.f, 0.f);
  };

  v4f acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  load(kt0);
  const int q = lane >> 4;  // which of the 4 real k of the MFMA k-slice
  for (uint64_t kt = kt0; kt < kt1; ++kt) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < A_LOADS; ++j)
      if (a_lds[j] >= 0) {
        As[a_lds[j]] = ra[j].x;
        As[a_lds[j] + SA] = ra[j].y;
      }
#pragma unroll
    for (int j = 0; j < B_LOADS; ++j)
      if (b_lds[j] >= 0) Bs[b_lds[j]] = rb[j];
    __syncthreads();
    if (kt + 1 < kt1) load(kt + 1);
#pragma unroll
    for (int kk = 0; kk < TK / WK; kk += 2) {
      const int ck = wk * (TK / WK) + kk + (q >> 1);
      const int part = q & 1;
      float av[BM], bv[BN];
#pragma unroll
      for (int bm = 0; bm < BM; ++bm) av[bm] = As[(2 * ck + part) * SA + (wm * BM + bm) * 16 + (lane & 15)];
#pragma unroll
      for (int bn = 0; bn < BN; ++bn) {
        const int col = lane & 15;
        float2 b = Bs[ck * SB + (wn * BN + bn) * 8 + (col >> 1)];
        float v = part == 0 ? ((col & 1) ? b.y : b.x) : ((col & 1) ? b.x : -b.y);
        bv[bn] = v;
      }
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn)
          acc[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[bm], bv[bn], acc[bm][bn], 0, 0, 0);
    }
  }
  __syncthreads();
  // Accumulators -> LDS tile (rows m, interleaved re/im columns).
  float* Cs = smem;
#pragma unroll
  for (int bm = 0; bm < BM; ++bm)
#pragma unroll
    for (int bn = 0; bn < BN; ++bn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int m = (wm * BM + bm) * 16 + 4 * (lane >> 4) + i;
        int col = (wn * BN + bn) * 16 + (lane & 15);
        Cs[(wk * TM + m) * SC + col] = acc[bm][bn][i];
      }
  __syncthreads();
  // LDS -> C, enumerated in C's address order.
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  const uint64_t baseC = scatter_bits(mt, d.cm + d.tm, d.mb - d.tm) + scatter_bits(nt, d.cn + d.tn, d.nb - d.tn) +
                         scatter_bits(batch, d.cb, d.bb);
  const int nc = d.tm + d.tn;
#pragma unroll
  for (int j = 0; j < C_ITEMS; ++j) {
    int e = tid + 256 * j;
    if (e >= (1 << nc)) break;
    uint32_t off = 0;
    int mi = 0, ni = 0;
    for (int b = 0; b < nc; ++b) {
      int bit = (e >> b) & 1;
      uint8_t code = d.c_tile[b];
      int idx = code & 31;
      if ((code >> 5) == TB_M) {
        mi |= bit << idx;
        off |= (uint32_t)bit << d.cm[idx];
      } else {
        ni |= bit << idx;
        off |= (uint32_t)bit << d.cn[idx];
      }
    }
    float2 v = make_float2(0.f, 0.f);
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      v.x += Cs[(w * TM + mi) * SC + 2 * ni];
      v.y += Cs[(w * TM + mi) * SC + 2 * ni + 1];
    }
    epilogue_store(d, baseC + off, v, blockIdx.y, c_elems);
  }
}

// Deterministic FP64 sum of split-K partials in split order (blocked
// summation, Sec. V-B / Eq. 3: each FP32 chain covers only K / splits terms).
__global__ __launch_bounds__(256) void k_reduce(StepDesc d) {
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  const uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= c_elems) return;
  const float2* part = reinterpret_cast<const float2*>(d.part);
  const uint64_t splits = 1ull << d.ks_bits;
  double sx = 0, sy = 0;
  for (uint64_t s = 0; s < splits; ++s) {
    float2 v = part[s * c_elems + c];
    sx += v.x;
    sy += v.y;
  }
  if (d.mode == EPI_ACC64) {
    double2* acc = reinterpret_cast<double2*>(d.acc);
    double2 o = acc[c];
    o.x += sx;
    o.y += sy;
    acc[c] = o;
  } else {
    reinterpret_cast<float2*>(d.C)[c] = make_float2((float)sx, (float)sy);
  }
}

// ---------------------------------------------------------------- launch
static hipError_t launch_stem(const StepDesc& d, dim3 grid, hipStream_t s) {
#define MITNC_STEM(KB, NB)                                              \
  if (d.kb == KB && d.nb == NB) {                                       \
    hipLaunchKernelGGL((k_stem<KB, NB>), grid, dim3(256), 0, s, d);     \
    return hipGetLastError();                                           \
  }
  MITNC_STEM(0, 0) MITNC_STEM(0, 1) MITNC_STEM(0, 2)
  MITNC_STEM(1, 0) MITNC_STEM(1, 1) MITNC_STEM(1, 2)
  MITNC_STEM(2, 0) MITNC_STEM(2, 1) MITNC_STEM(2, 2)
  MITNC_STEM(3, 0) MITNC_STEM(3, 1) MITNC_STEM(3, 2)
  MITNC_STEM(4, 0) MITNC_STEM(4, 1) MITNC_STEM(4, 2)
#undef MITNC_STEM
  return hipErrorInvalidValue;
}

hipError_t launch_step(int kclass, const StepDesc& d_in, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  StepDesc d = d_in;
  if (ev0) hipEventRecord(ev0, s);
  struct Rec {  // records ev1 right after the main kernel of the step
    hipEvent_t e;
    hipStream_t s;
    void operator()() const {
      if (e) hipEventRecord(e, s);
    }
  } rec{ev1, s};
  const uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
  switch (kclass) {
    case MITNC_K_SMALL: {
      dim3 grid((unsigned)((c_elems + 255) / 256));
      hipLaunchKernelGGL(k_small, grid, dim3(256), 0, s, d);
      rec();
      return hipGetLastError();
    }
    case MITNC_K_STEM: {
      int lowb = d.mb < 8 ? d.mb : 8;
      dim3 grid((unsigned)(1ull << (d.mb - lowb)), (unsigned)(1ull << d.bb));
      hipError_t e = launch_stem(d, grid, s);
      rec();
      return e;
    }
    case MITNC_K_TILE:
    case MITNC_K_TALL:
    case MITNC_K_SPLITK: {
      const int final_mode = d.mode;
      if (d.ks_bits > 0) d.mode = EPI_PARTIAL;
      dim3 grid((unsigned)(1ull << ((d.mb - d.tm) + (d.nb - d.tn))), (unsigned)(1ull << d.ks_bits),
                (unsigned)(1ull << d.bb));
      if (kclass == MITNC_K_TILE)
        hipLaunchKernelGGL((k_tile<2, 2, 1, 2, 4, 16>), grid, dim3(256), 0, s, d);
      else if (kclass == MITNC_K_TALL)
        hipLaunchKernelGGL((k_tile<4, 1, 1, 2, 2, 16>), grid, dim3(256), 0, s, d);
      else
        hipLaunchKernelGGL((k_tile<1, 1, 4, 1, 2, 64>), grid, dim3(256), 0, s, d);
      rec();
      hipError_t e = hipGetLastError();
      if (e != hipSuccess || d.ks_bits == 0) return e;
      d.mode = final_mode;
      hipLaunchKernelGGL(k_reduce, dim3((unsigned)((c_elems + 255) / 256)), dim3(256), 0, s, d);
      return hipGetLastError();
    }
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace mitnc
