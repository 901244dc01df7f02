// Descriptor of one pairwise contraction, passed by value to the kernels.
//
// The step computes C[b, m, n] = sum_k A[b, m, k] * B[b, k, n] over complex
// numbers, where m, n, k, b are "logical" coordinates whose bits are scattered
// over the address bits of each operand (the permutation of TTGT, Sec. II-A
// and V-A, applied as an address map instead of a copy).  Logical bit i of m
// sits at address bit am[i] of A and cm[i] of C, and so on.
#pragma once

#include <cstdint>

namespace mitnc {

enum EpilogueMode : int32_t {
  EPI_STORE = 0,    // C = result (complex64)
  EPI_ACC64 = 1,    // acc += result (complex128), used by the last step of a slice
  EPI_PARTIAL = 2,  // part[split][c address] = result; a reduction kernel finishes
};

// Tile-bit code: class in the top 3 bits (0 = m, 1 = k, 2 = n), logical bit
// index in the low 5 bits.
enum TileCls : uint8_t { TB_M = 0, TB_K = 1, TB_N = 2 };
inline constexpr uint8_t tile_code(int cls, int idx) { return (uint8_t)((cls << 5) | idx); }

struct StepDesc {
  const void* A;
  const void* B;
  void* C;
  double* acc;
  float* part;
  float* stats;            // optional per-step max |Re|,|Im| of stored outputs (float bits, atomicMax)
  int32_t mb, nb, kb, bb;  // bit counts of m, n, k, batch
  int32_t tm, tn, tk;      // tile bits (tiled kernels)
  int32_t ks_bits;         // K split over 2^ks_bits workgroups (high k bits)
  int32_t mode;            // EpilogueMode
  int32_t prec;            // storage of A, B, C: MITNC_C64, MITNC_CF16 or MITNC_CBF16
  int32_t step_index;      // slot in stats
  float out_scale;         // stored C = result * out_scale (a power of two)
  double acc_scale;        // EPI_ACC64: acc += result * acc_scale (a power of two)
  // Position tables; kernels copy them to LDS once (TAB_BYTES bytes from am).
  uint8_t am[32], ak[32], ab[32];
  uint8_t bk[32], bn[32], bbt[32];
  uint8_t cm[32], cn[32], cb[32];
  uint8_t a_tile[16], b_tile[16], c_tile[16];  // tile bits sorted by address position
  // FP16/BF16 tile kernels: the LDS word address of a tile entry is the XOR
  // of one vector per set tile bit (a GF(2)-linear map chosen per step for
  // conflict-free LDS access): row bit i of the A stage (m bit i) gives
  // ha_row[i], row bit r of the expanded B stage (r = 0: the re/im row of
  // the 2 x 2 block, r = i + 1: n bit i) gives hb_row[r], and tile k bit j
  // gives 1 << hk[j] (its column bit in the row).
  uint16_t ha_row[8], hb_row[8];
  uint8_t hk[8];
  // Complex64 tile kernels: LDS row k of the A (B) stage stores column m (n)
  // at m ^ H(k), H(k) the XOR of a_swz[j] (b_swz[j]) over the set bits j of
  // k.  Chosen per step so that the scattered staging writes and the
  // fragment reads hit distinct LDS banks (all zero: plain rows).
  uint8_t a_swz[8], b_swz[8];
  // FP16/BF16 tile kernels: 16-byte global loads wanted for A / B (the two
  // lowest tile bits are address bits 0 and 1); 4 or 1.
  uint8_t vec_a, vec_b;
};

// Byte offsets of the tables relative to StepDesc::am.
enum TabOff : int {
  T_AM = 0, T_AK = 32, T_AB = 64, T_BK = 96, T_BN = 128, T_BB = 160,
  T_CM = 192, T_CN = 224, T_CB = 256, T_ATILE = 288, T_BTILE = 304, T_CTILE = 320,
  T_HAROW = 336, T_HBROW = 352, T_HK = 368, TAB_BYTES = 376
};

// Device table entry mapping a single-qubit gate leaf's adjoint into the
// gradient accumulator (complex128, 4 entries U[out][in] per gate).
struct GradEntry {
  uint64_t adj_offset;           // byte offset of the leaf adjoint in the workspace
  int32_t gate;                  // index among single-qubit gates, circuit order
  int32_t rank;                  // unsliced bits of the leaf (0..2)
  int8_t full_pos[2];            // leaf address bit of each adjoint bit
  int8_t n_sliced;
  int8_t slice_bit[2];           // slice-id bit of each sliced leaf bit
  int8_t slice_pos[2];           // its leaf address bit
  int8_t pad_[7];
};

// Skinny split-K steps (complex64): at most 16 outputs per batch index and
// long K.  One wave per (k split, batch index); lanes take the six lowest k
// bits, each wave covers at least kSkinnyUnroll values of the higher ones.
inline constexpr int kSkinnyLaneBits = 6, kSkinnyUnroll = 4;
inline constexpr bool skinny_fits(int mb, int nb, int kb, int bb, int ks_bits) {
  return mb + nb <= 4 && kb >= kSkinnyLaneBits + 2 && ks_bits >= 0 && ks_bits <= kb - kSkinnyLaneBits - 2 &&
         bb <= 16;
}

// SMALL steps within the class limits (at most 2^10 outputs, K <= 64) take
// the small kernel's bounded, branch-free address code.
inline constexpr int kSmallBits = 10;
inline constexpr bool small_bounded(int mb, int nb, int kb, int bb) {
  return mb <= kSmallBits && nb <= kSmallBits && bb <= kSmallBits && kb <= 6;
}

// One SMALL-class adjoint contraction of the reverse pass inside a batched
// launch (device table in the workspace).  The descriptor gives the shape and
// position tables; operands are workspace byte offsets, and the one operand
// that may be a leaf with sliced indices gets its slice offset in the kernel.
struct SmallRevOp {
  StepDesc d;                    // A, B, C unused
  uint64_t a_off, b_off, c_off;  // workspace byte offsets of A, B, C
  uint32_t block0;               // index of the op's first workgroup in the block table
  int8_t sl_which;               // 0: none, 1: A, 2: B is a leaf with sliced indices
  int8_t sl_n;                   // its sliced indices (at most 8)
  int8_t sl_bit[8];              // slice-id bit of each
  int8_t sl_pos[8];              // its leaf address bit
  int8_t pad_[6];
};

// One step of the batched range prologue (forward steps a slice range
// computes once): operands and output are workspace byte offsets; an operand
// with sliced indices (all constant over the range) is read at entry offset
// sum_j ((slice >> bit[j]) & 1) << pos[j].
struct SmallFwdOp {
  StepDesc d;                    // A, B, C, stats unused
  uint64_t a_off, b_off, c_off;
  uint32_t block0;               // index of the op's first workgroup in the block table
  int8_t na, nb;                 // sliced indices of A and B (at most 16 each)
  int8_t a_bit[16], a_pos[16], b_bit[16], b_pos[16];
  int8_t pad_[2];
};

// Tile geometry of the MFMA kernel classes (bits of the m, n, k tile).
struct TileGeom {
  int tm_bits, tn_bits, tk_bits;
};
// Wave layout of the square-tile kernels (TILE class): WM x WN x WK waves,
// BM x BN MFMA blocks per wave, TK complex k per k tile.  Compile-time
// constants (overridable with -D for tuning builds); the plan's tile bits
// follow from them.
#ifndef MITNC_TILE_WM
#define MITNC_TILE_WM 4
#define MITNC_TILE_WN 1
#define MITNC_TILE_WK 1
#define MITNC_TILE_BM 2
#define MITNC_TILE_BN 4
#define MITNC_TILE_TK 8
#endif
#ifndef MITNC_TILEH_WM
#define MITNC_TILEH_WM 2
#define MITNC_TILEH_WN 2
#define MITNC_TILEH_WK 1
#define MITNC_TILEH_BM 4
#define MITNC_TILEH_BN 4
#define MITNC_TILEH_TK 32
#endif
inline constexpr int ilog2_exact(int x) { return x <= 1 ? 0 : 1 + ilog2_exact(x >> 1); }
// complex64 (3M split on FP32 MFMA): 16 x 16 MFMA blocks
inline constexpr TileGeom geom_tile() {
  return {ilog2_exact(MITNC_TILE_WM * MITNC_TILE_BM * 16), ilog2_exact(MITNC_TILE_WN * MITNC_TILE_BN * 16),
          ilog2_exact(MITNC_TILE_TK)};
}
inline constexpr TileGeom geom_tall() { return {7, 4, 4}; }    // 128 x 16, k 16
inline constexpr TileGeom geom_splitk() { return {4, 4, 6}; }  // 16 x 16, k 64 (4 waves split k)
// complex FP16 / BF16 (4M split on 16x16x32 MFMA)
inline constexpr TileGeom geom_tile_h() {  // 16 rows x 8 complex columns per MFMA block
  return {ilog2_exact(MITNC_TILEH_WM * MITNC_TILEH_BM * 16), ilog2_exact(MITNC_TILEH_WN * MITNC_TILEH_BN * 8),
          ilog2_exact(MITNC_TILEH_TK)};
}
inline constexpr TileGeom geom_tall_h() { return {7, 4, 5}; }    // 128 x 16, k 32
inline constexpr TileGeom geom_splitk_h() { return {4, 4, 7}; }  // 16 x 16, k 128 (4 waves split k)

// Fused stem section (Sec. IV): a chain of steps on one large tensor T, each
// contracting T with a small matrix, run as one kernel.  A workgroup loads a
// tile of T (its intra-tile bits: every bit the section contracts, plus low
// address bits for coalescing) into LDS, applies the steps there and writes
// the final tile; the other (inter-tile) bits only select the tile.
inline constexpr int kMaxSectionSteps = 8;
inline constexpr int kSectionClass = 6;    // timing slot of fused sections
inline constexpr int kMaxTileBits = 13;    // 2^13 complex entries = 64 KB per LDS buffer
inline constexpr int kTileBitsTarget = 12; // sections prefer 2^12-entry tiles (two workgroups per CU)
inline constexpr int kMaxSectionB = 1024;  // padded B entries per step
inline constexpr unsigned kSectionMaxLds = 160u * 1024u - 2048u;  // dynamic LDS bytes of a section kernel
struct TileStep {
  const void* B;       // small operand, storage of the run's precision
  int32_t mb, kb, nb;  // tile bits kept (m), contracted (k), new (n)
  int32_t step_index;  // plan step (statistics slot)
  float out_scale;     // FP16/BF16: 2^(eA + eB - eC); 1 for complex64
  uint32_t b_lds;      // float2 offset of the step's padded B^T in LDS
  uint32_t kpad;       // row length of the padded B^T (max(K, 4))
  uint8_t am[16];      // input LDS buffer bit of each m bit (bits 0-3 ride on lanes)
  uint8_t ak[8];       // input LDS buffer bit of each k bit (bits 0-1 ride on lanes)
  uint8_t cm[16];      // output LDS buffer bit of each m bit
  uint8_t cn[8];       // output LDS buffer bit of each n bit
  uint8_t bk[8], bn[8];  // B address bits of k and n
};
struct SectionDesc {
  const void* A;       // T at the section's start
  void* C;             // T at its end
  float* stats;        // optional per-step maxima (as StepDesc::stats)
  int32_t prec;
  int32_t n_steps;
  int32_t t_in, t_out;     // tile bits at start and end
  int32_t outer_bits;      // inter-tile bits (the same labels in A and C)
  int32_t tile_max;        // LDS buffer size in entries (power of two): tb tiles
  int32_t tb_bits;         // log2 of the tiles processed together (a tile group)
  int32_t stride_bits;     // log2 of a tile's slot in a buffer (largest tile of the section)
  uint32_t b_total;        // float2 entries of all B^T copies
  uint8_t p_in[16];        // A address bit of tile bit i (ascending)
  uint8_t p_out[16];       // C address bit of tile bit i of the final buffer (ascending)
  uint8_t q_in[32];        // A address bit of outer bit i
  uint8_t q_out[32];       // C address bit of outer bit i
  TileStep st[kMaxSectionSteps];
};

// Stream class limits: at most 2^10 batch indices, at least 2^8 rows, K, N
// <= 64 and at most 16 (k step, column block) pairs of B held in registers
// per lane.
inline constexpr int kStreamMinM = 8;
inline constexpr bool stream_fits(int mb, int nb, int kb, int bb) {
  return bb <= 10 && mb >= kStreamMinM && kb <= 6 && nb <= 6 && (kb > 2 ? kb - 2 : 0) + (nb > 4 ? nb - 4 : 0) <= 4;
}

// The stream kernels address a lane's entries as a scalar 64-bit base (row
// block, batch, and the k or n bits that are the same on every lane of a
// wave) plus a 32-bit byte offset that holds only the lane-varying bits: the
// four lowest row bits and the lowest k bits (two for complex64 entries,
// three for 16-bit ones) in A, the four lowest row bits and the two lowest n
// bits in C.  Those bits' largest offset must stay below 4 GiB at the entry
// sizes (A, C or the FP64 result) the launch uses.
inline bool stream_offsets_fit(const StepDesc& d, uint64_t a_bytes, uint64_t c_bytes) {
  uint64_t a = 0, c = 0;
  auto add = [](uint64_t& m, const uint8_t* pos, int n) {
    for (int i = 0; i < n; ++i) {
      if (pos[i] >= 40) return false;
      m |= 1ull << pos[i];
    }
    return true;
  };
  const int lanes = d.mb < 4 ? d.mb : 4;
  const int k_lane = a_bytes == 8 ? 2 : 3;
  if (!add(a, d.am, lanes) || !add(a, d.ak, d.kb < k_lane ? d.kb : k_lane) || !add(c, d.cm, lanes) ||
      !add(c, d.cn, d.nb < 2 ? d.nb : 2))
    return false;
  return a * a_bytes < (1ull << 32) && c * c_bytes < (1ull << 32);
}

// The stream kernel steps C's rows with the same scattered-bit increment as
// A's, so the row bits above the four lane bits must ascend in C as in A.
inline bool stream_rows_sorted(const StepDesc& d) {
  for (int i = 5; i < d.mb; ++i)
    if (d.cm[i] <= d.cm[i - 1]) return false;
  return true;
}

}  // namespace mitnc
