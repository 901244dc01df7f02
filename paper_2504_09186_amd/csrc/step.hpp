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
  const float* A;
  const float* B;
  float* C;
  double* acc;
  float* part;
  int32_t mb, nb, kb, bb;  // bit counts of m, n, k, batch
  int32_t tm, tn, tk;      // tile bits (tiled kernels)
  int32_t ks_bits;         // K split over 2^ks_bits workgroups (high k bits)
  int32_t mode;            // EpilogueMode
  int32_t pad_;
  uint8_t am[32], ak[32], ab[32];
  uint8_t bk[32], bn[32], bbt[32];
  uint8_t cm[32], cn[32], cb[32];
  uint8_t a_tile[16], b_tile[16], c_tile[16];  // tile bits sorted by address position
};

// Tile geometry of the MFMA kernel classes.
struct TileGeom {
  int tm_bits, tn_bits, tk_bits;
};
inline constexpr TileGeom geom_tile() { return {6, 6, 4}; }    // 64 x 64 complex, k 16
inline constexpr TileGeom geom_tall() { return {7, 4, 4}; }    // 128 x 16, k 16
inline constexpr TileGeom geom_splitk() { return {4, 4, 6}; }  // 16 x 16, k 64 (4 waves split k)

}  // namespace mitnc
