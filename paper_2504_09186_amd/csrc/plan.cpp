// Plan construction: layouts, kernel classes, reuse levels and memory.
//
//  * Layouts (Sec. V-A): a rank-r tensor is a flat array whose address bits
//    are its binary indices.  The permutation that brings the common indices
//    together is never materialised; each step carries, for every operand,
//    the address bit of every logical m/n/k/batch bit, and the kernels stage
//    tiles through LDS with that map.  The output layout is free: the new
//    indices of the small operand take the address bits freed by the
//    contracted indices of the large one, so a stem tensor keeps its layout
//    from step to step.  The larger operand is always "A" (Sec. V-A: keep the
//    large tensor as the multiplier).
//  * Reuse (Sec. III-B, tree-like pre-lifetime reuse): slices are run in
//    slice-id order, the last sliced index fastest.  A node depends on the
//    slice-id bits of the sliced indices in its subtree; between slice s-1 and
//    s the bits 0..ctz(s) change, so a node is recomputed iff its lowest
//    dependency bit is <= ctz(s).  A node recomputed less often than its parent
//    is kept across slices (one stored tensor per fork).
//  * Kernel classes: tiny steps, stream steps (a big tensor times a small
//    matrix on MFMA, HBM bound), stem steps (the same on vector FMA, for
//    batched or short ones), square-ish GEMM tiles on MFMA, narrow tiles, and
//    split-K for K >> M, N (Sec. V-B, split-common TTGT).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <tuple>

#include "plan.hpp"

namespace mitnc {

static uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Split-K: every split keeps more than 2^kSplitMinStageBits k tiles.
#ifndef MITNC_SPLIT_MIN_STAGE_BITS
#define MITNC_SPLIT_MIN_STAGE_BITS 2
#endif
static constexpr int kSplitMinStageBits = MITNC_SPLIT_MIN_STAGE_BITS;
// Split-K workgroup targets (log2) of the TILE and TALL classes.
#ifndef MITNC_TILE_SPLIT_TARGET
#define MITNC_TILE_SPLIT_TARGET 9
#endif
#ifndef MITNC_TALL_SPLIT_TARGET
#define MITNC_TALL_SPLIT_TARGET 9
#endif

static void fill_positions(uint8_t* dst, const std::vector<int>& src) {
  for (size_t i = 0; i < src.size(); ++i) dst[i] = (uint8_t)src[i];
}

// Tile bits of one operand sorted by address position.  Each entry is
// (position, code).
static void tile_order(uint8_t* dst, std::vector<std::pair<int, uint8_t>> v) {
  std::sort(v.begin(), v.end());
  for (size_t i = 0; i < v.size(); ++i) dst[i] = v[i].second;
}

namespace {
// Span of a set of vectors over GF(2) (bit b of piv[b] is its leading bit).
struct XorSpan {
  uint32_t piv[32] = {};
  bool contains(uint32_t v) const {  // true for v == 0
    for (int b = 31; b >= 0; --b)
      if ((v >> b) & 1) {
        if (!piv[b]) return false;
        v ^= piv[b];
      }
    return true;
  }
  void add(uint32_t v) {
    for (int b = 31; b >= 0; --b)
      if ((v >> b) & 1) {
        if (!piv[b]) {
          piv[b] = v;
          return;
        }
        v ^= piv[b];
      }
  }
};
}  // namespace

// Row XOR masks of a complex64 tile operand in LDS: rows are the k bits,
// 2^col_bits float2 columns per row, no padding; row k stores column c at
// c ^ H(k), H(k) the XOR of g[j] over the set bits j of k (g[j] < 2^col_bits).
// A float2 slot covers two 4-byte banks, so a wave access is served 16 lanes
// (32 banks) or 32 lanes (64 banks) at a time and is conflict-free when those
// lanes' slots differ mod 16 (mod 32).  Staging writes: lanes take
// consecutive tile elements in address order, so lanes 0-15 (0-31) differ in
// the tile bits codes[0..3] (codes[0..4]); the slot moves by 2^i for column
// bit i and by 2^(col_bits + j) ^ g[j] for row bit j, and the writes are
// conflict-free when those moves are linearly independent (GF(2)) mod 16 and
// mod 32.  The g of the row bits among the lowest tile bits are chosen in
// that order to keep both sets independent.  Fragment reads take 16
// consecutive columns of one row per 16 lanes (a permutation of 16
// consecutive slots) and rows k, k + 1 in lanes 0-31: g[0] gets bit 4 where
// free, so those two rows use the two halves of 64 banks.
static void lds_row_swizzle(const uint8_t* codes, int ncodes, int row_cls, int col_bits, uint8_t* g) {
  std::fill(g, g + 8, (uint8_t)0);
  const uint32_t cols = 1u << col_bits;
  const uint32_t gmax = cols < 32 ? cols : 32;
  auto colvec = [](int i) -> uint32_t { return i < 5 ? 1u << i : 0u; };
  const int nl = ncodes < 5 ? ncodes : 5;
  XorSpan s16, s32;
  for (int t = 0; t < nl; ++t) {
    if ((codes[t] >> 5) == row_cls) continue;
    const uint32_t v = colvec(codes[t] & 31);
    if (t < 4) s16.add(v & 15);
    s32.add(v);
  }
  bool row0_lane = false;
  for (int t = 0; t < nl; ++t) {
    if ((codes[t] >> 5) != row_cls) continue;
    const int j = codes[t] & 31;
    if (j >= 8) continue;
    const uint32_t stride = (cols << j) & 31;
    if (j == 0) row0_lane = true;
    std::vector<uint32_t> cand;
    for (uint32_t v = 0; v < gmax; ++v) cand.push_back(v);
    auto key = [&](uint32_t v) {
      const int hi = (j == 0 && ((stride ^ v) & 16)) ? 0 : 1;
      return std::make_tuple(hi, __builtin_popcount(v), v);
    };
    std::sort(cand.begin(), cand.end(), [&](uint32_t a, uint32_t b) { return key(a) < key(b); });
    int pick = -1;
    for (int pass = 0; pass < 2 && pick < 0; ++pass)
      for (uint32_t v : cand) {
        const uint32_t vec = stride ^ v;
        const bool ok16 = t > 3 || !s16.contains(vec & 15);
        const bool ok32 = !s32.contains(vec);
        if (ok16 && (ok32 || pass == 1)) {
          pick = (int)v;
          break;
        }
      }
    if (pick < 0) pick = 0;
    g[j] = (uint8_t)pick;
    const uint32_t vec = stride ^ (uint32_t)pick;
    if (t < 4) s16.add(vec & 15);
    s32.add(vec);
  }
  if (!row0_lane && gmax == 32 && !(cols & 16)) g[0] = 16;
}

// ---------------------------------------------------------------- FP16/BF16 tile LDS layout
// The FP16/BF16 tile kernels keep A as TM rows (m) and the expanded B as
// 2 TN rows (2n + re/im) of 2^tkb 32-bit words (one complex k per word).
// The word address of a tile entry is the XOR of one vector per set bit:
// m bit i -> ha_row[i], B row bit r -> hb_row[r], k bit j -> 1 << hk[j].
// Row vectors are the row stride plus a swizzle c << 2 (c permutes the
// 4-word groups of a row), so the map is a bijection and 4-word groups stay
// contiguous for the 16-byte fragment reads.
//
// Bank model: 4-byte banks, 32 (128 B per clock) or 64 (256 B per clock);
// a wave access is served in groups of lanes that together fill the banks
// once (32 lanes for 4-byte, 8 for 16-byte accesses with 32 banks; twice as
// many with 64), and a group whose lanes differ in d address bits that are
// linearly dependent over GF(2) in the bank index takes 2^d times as long.
namespace {
struct HDesign {
  uint16_t arow[8] = {}, brow[8] = {};
  uint8_t hk[8] = {};
  int va = 1, vb = 1;
  double cost = 1e30;
};

int gf2_rank(const uint32_t* v, int n) {
  XorSpan s;
  int r = 0;
  for (int i = 0; i < n; ++i)
    if (!s.contains(v[i])) {
      s.add(v[i]);
      ++r;
    }
  return r;
}

// Modeled cycles of one 64-lane LDS access whose lane bits 0..5 move the
// word address by lane_vec[0..5], width 1 or 4 words, summed over the
// 32- and 64-bank models.
double access_cost(const uint32_t* lane_vec, int width) {
  double c = 0;
  for (int nb : {32, 64}) {
    const int per = nb / width;  // lanes per group
    const int L = __builtin_ctz(per);
    const int sh = width == 4 ? 2 : 0;
    uint32_t v[6];
    for (int i = 0; i < L; ++i) v[i] = (lane_vec[i] >> sh) & (uint32_t)(per - 1);
    const int deg = 1 << (L - gf2_rank(v, L));
    c += (64.0 / per) * deg;  // groups per instruction x conflict degree
  }
  return c;
}

// Row swizzles c0..c3 (of row bits 0..3) for which 16-byte fragment reads
// of 8 (16) consecutive rows hit distinct 4-word blocks mod 32 (64) banks.
const std::vector<std::array<uint8_t, 4>>& read_feasible(int tkb) {
  static std::vector<std::array<uint8_t, 4>> cache[16];
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  auto& f = cache[tkb];
  if (!f.empty()) return f;
  const int ng = std::min(tkb - 2, 4);
  const int G = 1 << ng;
  for (int c0 = 0; c0 < G; ++c0)
    for (int c1 = 0; c1 < G; ++c1)
      for (int c2 = 0; c2 < G; ++c2)
        for (int c3 = 0; c3 < G; ++c3) {
          const int cs[4] = {c0, c1, c2, c3};
          uint32_t r32[3], r64[4];
          for (int i = 0; i < 4; ++i) {
            const uint32_t rv = (1u << (i + tkb)) ^ ((uint32_t)cs[i] << 2);
            if (i < 3) r32[i] = (rv >> 2) & 7;
            r64[i] = (rv >> 2) & 15;
          }
          if (gf2_rank(r32, 3) == 3 && gf2_rank(r64, 4) == 4)
            f.push_back({(uint8_t)c0, (uint8_t)c1, (uint8_t)c2, (uint8_t)c3});
        }
  return f;
}

// Best row vectors for one operand: codes = tile bits in address order,
// row_cls = class of the row bits, row_off = row bit of row index 0 of that
// class (1 for the expanded B), nrows = template row bits.  Returns the cost
// of the operand's staging writes per k tile and thread.
double choose_rows(const uint8_t* codes, int ncodes, int row_cls, int row_off, int nrows, int tkb,
                   const uint8_t* hk, int vec, int words_per_thread, int copies, uint16_t* rows_out) {
  const auto& feas = read_feasible(tkb);
  const int ub = vec == 4 ? 2 : 0;
  double best = 1e30;
  for (const auto& cs : feas) {
    uint32_t rv[8];
    for (int i = 0; i < nrows; ++i) rv[i] = (1u << (i + tkb)) ^ (i < 4 ? (uint32_t)cs[i] << 2 : 0u);
    auto vec_of = [&](uint8_t code) -> uint32_t {
      const int cls = code >> 5, idx = code & 31;
      if (cls == row_cls) return rv[idx + row_off];
      return 1u << hk[idx];
    };
    uint32_t lane[6] = {};
    for (int i = 0; i < 6; ++i) lane[i] = ub + i < ncodes ? vec_of(codes[ub + i]) : 0u;
    const bool contig = vec == 4 && ncodes >= 2 && vec_of(codes[0]) == 1 && vec_of(codes[1]) == 2;
    const double per_instr = contig ? access_cost(lane, 4) : access_cost(lane, 1);
    const int instr = contig ? std::max(1, words_per_thread / 4) : std::max(1, words_per_thread);
    const double cost = per_instr * instr * copies;
    if (cost < best) {
      best = cost;
      for (int i = 0; i < nrows; ++i) rows_out[i] = (uint16_t)rv[i];
    }
  }
  return best;
}
}  // namespace

// Chooses the FP16/BF16 tile LDS layout of a step (see above): 16-byte
// loads for each operand whose layout allows them, and among k-bit orders
// that put the lowest k bits of A or B at columns 0 and 1, the one with the
// fewest modeled staging-write cycles (reads are conflict-free by
// construction).
static void lds_design_h(StepDesc& d, const TileGeom& g) {
  const int tkb = g.tk_bits;
  auto pos_a = [&](uint8_t c) { return (c >> 5) == TB_M ? d.am[c & 31] : d.ak[c & 31]; };
  auto pos_b = [&](uint8_t c) { return (c >> 5) == TB_K ? d.bk[c & 31] : d.bn[c & 31]; };
  const int na = d.tm + d.tk, nb = d.tk + d.tn;
  const bool va_ok = na >= 2 && pos_a(d.a_tile[0]) == 0 && pos_a(d.a_tile[1]) == 1;
  const bool vb_ok = nb >= 2 && pos_b(d.b_tile[0]) == 0 && pos_b(d.b_tile[1]) == 1;
  // The choice depends only on the tile codes, the load-width conditions
  // and the geometry: repeated shapes (one-step contractions, plans built
  // again) take it from a cache.
  std::string key(reinterpret_cast<const char*>(d.a_tile), (size_t)na);
  key.append(reinterpret_cast<const char*>(d.b_tile), (size_t)nb);
  key += {(char)na, (char)nb, (char)va_ok, (char)vb_ok, (char)g.tm_bits, (char)g.tn_bits, (char)tkb};
  static std::mutex cache_mu;
  static std::map<std::string, HDesign> cache;
  auto apply = [&](const HDesign& h) {
    std::memcpy(d.ha_row, h.arow, sizeof d.ha_row);
    std::memcpy(d.hb_row, h.brow, sizeof d.hb_row);
    std::memcpy(d.hk, h.hk, sizeof d.hk);
    d.vec_a = (uint8_t)h.va;
    d.vec_b = (uint8_t)h.vb;
  };
  {
    std::lock_guard<std::mutex> lk(cache_mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      apply(it->second);
      return;
    }
  }
  std::vector<int> ka, kb;  // tile k bits in address order
  for (int i = 0; i < na; ++i)
    if ((d.a_tile[i] >> 5) == TB_K) ka.push_back(d.a_tile[i] & 31);
  for (int i = 0; i < nb; ++i)
    if ((d.b_tile[i] >> 5) == TB_K) kb.push_back(d.b_tile[i] & 31);
  std::vector<std::vector<int>> firsts;
  auto two = [](const std::vector<int>& v) { return std::vector<int>(v.begin(), v.begin() + std::min<size_t>(2, v.size())); };
  firsts.push_back(two(ka));
  firsts.push_back(two(kb));
  if (!ka.empty() && !kb.empty()) {
    for (int x : kb)
      if (x != ka[0]) {
        firsts.push_back({ka[0], x});
        break;
      }
    for (int x : ka)
      if (x != kb[0]) {
        firsts.push_back({kb[0], x});
        break;
      }
  }
  firsts.push_back({});
  const int wa = std::max(1, (1 << na) / 256), wb = std::max(1, (1 << nb) / 256);
  const int nrow_a = g.tm_bits, nrow_b = g.tn_bits + 1;
  HDesign best;
  std::set<std::vector<int>> seen;
  for (const auto& f : firsts) {
    if (!seen.insert(f).second) continue;
    uint8_t hk[8] = {};
    std::vector<char> used(8, 0);
    int col = 0;
    for (int j : f) {
      hk[j] = (uint8_t)col++;
      used[j] = 1;
    }
    for (int j = 0; j < d.tk; ++j)
      if (!used[j]) hk[j] = (uint8_t)col++;
    for (int va : {4, 1}) {
      if (va == 4 ? !va_ok : va_ok) continue;  // 16-byte loads whenever the layout has them
      uint16_t ra[8] = {};
      const double ca = choose_rows(d.a_tile, na, TB_M, 0, nrow_a, tkb, hk, va, wa, 1, ra);
      for (int vb : {4, 1}) {
        if (vb == 4 ? !vb_ok : vb_ok) continue;
        uint16_t rb[8] = {};
        const double cb = choose_rows(d.b_tile, nb, TB_N, 1, nrow_b, tkb, hk, vb, wb, 2, rb);
        const double cost = ca + cb - 1e-3 * (va + vb);  // ties: wider loads
        if (cost < best.cost) {
          best.cost = cost;
          best.va = va;
          best.vb = vb;
          std::memcpy(best.arow, ra, sizeof ra);
          std::memcpy(best.brow, rb, sizeof rb);
          std::memcpy(best.hk, hk, sizeof hk);
        }
      }
    }
  }
  apply(best);
  std::lock_guard<std::mutex> lk(cache_mu);
  if (cache.size() > 4096) cache.clear();
  cache.emplace(key, best);
}

static TileGeom geom_of(int kclass, int precision) {
  const bool h = precision != MITNC_C64;
  switch (kclass) {
    case MITNC_K_TILE: return h ? geom_tile_h() : geom_tile();
    case MITNC_K_TALL: return h ? geom_tall_h() : geom_tall();
    case MITNC_K_SPLITK: return h ? geom_splitk_h() : geom_splitk();
    default: return {0, 0, 0};
  }
}

// 16-bit storage of a complex entry (re in the low half).
static uint32_t host_f16(float f) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f); }
static uint32_t host_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// Exponent e so that max * 2^-e lies in [2^13, 2^14): two bits of headroom
// below the FP16 maximum (65504) for slice-to-slice variation.
int mantissa_exponent(double max_abs) {
  if (!(max_abs > 0) || !std::isfinite(max_abs)) return 0;
  int e2;
  std::frexp(max_abs, &e2);  // max = f * 2^e2, f in [0.5, 1)
  return (e2 - 1) - 13;
}

// Split-K takes steps whose m and n bit counts are both at most `smn`
// (plan option; 4 by default: M, N <= 16, Sec. V-B's narrow GEPDOTs).
static int splitk_mn_bits(const mitnc_plan* P) {
  const int v = P->opts.splitk_max_mn_bits;
  return v > 0 ? std::min(v, 8) : 4;
}

static int choose_class_no_stream(int mb, int nb, int kb, int bb, int smn) {
  if (mb + nb + bb <= 10 && kb <= 6) return MITNC_K_SMALL;
  if (nb <= 2 && kb <= 4) return MITNC_K_STEM;
  if (mb <= smn && nb <= smn) return MITNC_K_SPLITK;
  if (nb <= 4) return MITNC_K_TALL;
  return MITNC_K_TILE;
}

static int choose_class(int mb, int nb, int kb, int bb, int smn) {
  int out_bits = mb + nb + bb;
  if (out_bits <= 10 && kb <= 6) return MITNC_K_SMALL;
  if (stream_fits(mb, nb, kb, bb)) return MITNC_K_STREAM;
  if (nb <= 2 && kb <= 4) return MITNC_K_STEM;
  if (mb <= smn && nb <= smn) return MITNC_K_SPLITK;
  if (nb <= 4) return MITNC_K_TALL;
  return MITNC_K_TILE;
}

// True when the row indices M (sorted by A position) above the lowest four
// also come in ascending position in the output layout C.
static bool rows_in_order(const std::vector<int64_t>& M, const std::vector<int64_t>& C) {
  std::map<int64_t, int> pc;
  for (size_t i = 0; i < C.size(); ++i) pc[C[i]] = (int)i;
  for (size_t i = 5; i < M.size(); ++i)
    if (pc[M[i]] <= pc[M[i - 1]]) return false;
  return true;
}

// Builds the descriptor of a step given the operand layouts.
static void build_step(mitnc_plan* P, PlanStep& st, const std::vector<int64_t>& c_labels_set,
                       const std::vector<int64_t>* root_layout, int force_kernel, int precision) {
  PlanNode& A0 = P->nodes[st.a];
  PlanNode& B0 = P->nodes[st.b];
  std::map<int64_t, int> pa, pb, inC;
  for (size_t i = 0; i < A0.labels.size(); ++i) pa[A0.labels[i]] = A0.pos[i];
  for (size_t i = 0; i < B0.labels.size(); ++i) pb[B0.labels[i]] = B0.pos[i];
  for (int64_t x : c_labels_set) inC[x] = 1;
  if (B0.rank > A0.rank) {
    std::swap(st.a, st.b);
    std::swap(pa, pb);
    st.swapped = true;
  }
  PlanNode& A = P->nodes[st.a];
  PlanNode& B = P->nodes[st.b];
  std::vector<int64_t> M, N, K, Bt;
  for (auto& [x, p] : pa) {
    bool b = pb.count(x), c = inC.count(x);
    if (b && c) Bt.push_back(x);
    else if (b) K.push_back(x);
    else if (c) M.push_back(x);
    else fail(MITNC_UNSUPPORTED, "index held by one operand only and not kept");
  }
  for (auto& [x, p] : pb) {
    if (pa.count(x)) continue;
    if (!inC.count(x)) fail(MITNC_UNSUPPORTED, "index held by one operand only and not kept");
    N.push_back(x);
  }
  auto by = [](std::map<int64_t, int>& m) { return [&m](int64_t u, int64_t v) { return m[u] < m[v]; }; };
  std::sort(M.begin(), M.end(), by(pa));
  std::sort(N.begin(), N.end(), by(pb));
  std::sort(Bt.begin(), Bt.end(), by(pa));
  int kclass = force_kernel >= 0 ? force_kernel
                                 : choose_class((int)M.size(), (int)N.size(), (int)K.size(), (int)Bt.size(), splitk_mn_bits(P));
  if (force_kernel < 0 && kclass == MITNC_K_STREAM && root_layout && !rows_in_order(M, *root_layout))
    kclass = choose_class_no_stream((int)M.size(), (int)N.size(), (int)K.size(), (int)Bt.size(), splitk_mn_bits(P));
  if (kclass == MITNC_K_STREAM) {
    // Stream kernel: the two lowest k bits ride on lanes next to the four
    // lowest m bits, so K goes by A position (B is small and cached).
    std::sort(K.begin(), K.end(), by(pa));
  } else {
    // K order: indices among the lowest 4 address bits of A or B first (they
    // must be inside every tile for coalesced loads), then by A position.
    std::sort(K.begin(), K.end(), [&](int64_t u, int64_t v) {
      int lu = std::min(pa[u], pb[u]) < 4 ? 0 : 1, lv = std::min(pa[v], pb[v]) < 4 ? 0 : 1;
      if (lu != lv) return lu < lv;
      if (lu == 0) return std::min(pa[u], pb[u]) < std::min(pa[v], pb[v]);
      return pa[u] < pa[v];
    });
  }
  // Output layout.
  std::vector<int64_t> C;
  if (root_layout) {
    C = *root_layout;
  } else {
    std::vector<std::pair<int, int64_t>> order;
    for (auto& [x, p] : pa) order.push_back({p, x});
    std::sort(order.begin(), order.end());
    size_t ni = 0;
    std::map<int64_t, char> isK;
    for (auto x : K) isK[x] = 1;
    for (auto& [p, x] : order) {
      if (isK.count(x)) {
        if (ni < N.size()) C.push_back(N[ni++]);
      } else {
        C.push_back(x);  // M or batch
      }
    }
    while (ni < N.size()) C.push_back(N[ni++]);
  }
  std::map<int64_t, int> pc;
  for (size_t i = 0; i < C.size(); ++i) pc[C[i]] = (int)i;
  if (C.size() != M.size() + N.size() + Bt.size()) fail(MITNC_UNSUPPORTED, "output label mismatch");

  PlanNode& O = P->nodes[st.out];
  O.labels = C;
  O.pos.resize(C.size());
  std::iota(O.pos.begin(), O.pos.end(), 0);
  O.rank = (int)C.size();
  O.full_rank = O.rank;

  StepDesc& d = st.d;
  std::memset(&d, 0, sizeof(d));
  d.mb = (int)M.size();
  d.nb = (int)N.size();
  d.kb = (int)K.size();
  d.bb = (int)Bt.size();
  if (d.mb > 32 || d.nb > 32 || d.kb > 32 || d.bb > 32) fail(MITNC_UNSUPPORTED, "rank too large");
  std::vector<int> v;
  auto put = [&](uint8_t* dst, const std::vector<int64_t>& ls, std::map<int64_t, int>& m) {
    v.clear();
    for (auto x : ls) v.push_back(m[x]);
    fill_positions(dst, v);
  };
  put(d.am, M, pa);
  put(d.ak, K, pa);
  put(d.ab, Bt, pa);
  put(d.bk, K, pb);
  put(d.bn, N, pb);
  put(d.bbt, Bt, pb);
  put(d.cm, M, pc);
  put(d.cn, N, pc);
  put(d.cb, Bt, pc);

  st.kclass = kclass;
  if (st.kclass < MITNC_K_SMALL || st.kclass > MITNC_K_STREAM) fail(MITNC_INVALID_ARG, "unknown kernel class");
  if (st.kclass == MITNC_K_STEM && (d.kb > 4 || d.nb > 2))
    fail(MITNC_UNSUPPORTED, "stem kernel needs at most 4 contracted and 2 new indices");
  // Lane offsets of the stream kernels are 32-bit byte offsets (sized for
  // the FP64 result, the largest entry an output may get).
  const uint64_t stream_a_bytes = precision == MITNC_C64 ? 8 : 4;
  if (st.kclass == MITNC_K_STREAM && force_kernel < 0 && !stream_offsets_fit(d, stream_a_bytes, 16))
    return build_step(P, st, c_labels_set, root_layout, choose_class_no_stream(d.mb, d.nb, d.kb, d.bb, splitk_mn_bits(P)),
                      precision);
  if (st.kclass == MITNC_K_STREAM &&
      (!stream_fits(d.mb, d.nb, d.kb, d.bb) || !stream_rows_sorted(d) || !stream_offsets_fit(d, stream_a_bytes, 16)))
    fail(MITNC_UNSUPPORTED,
         "stream kernel needs <= 10 batch bits, >= 8 row bits, K, N <= 64, K N / 64 <= 16, C row bits in order "
         "and lane offsets below 4 GiB");
  TileGeom g = geom_of(st.kclass, precision);
  d.prec = precision;
  d.out_scale = 1.f;
  d.acc_scale = 1.0;
  d.tm = std::min(g.tm_bits, d.mb);
  d.tn = std::min(g.tn_bits, d.nb);
  d.tk = std::min(g.tk_bits, d.kb);
  if (st.kclass == MITNC_K_TILE || st.kclass == MITNC_K_TALL || st.kclass == MITNC_K_SPLITK) {
    std::vector<std::pair<int, uint8_t>> ta, tb, tc;
    for (int i = 0; i < d.tm; ++i) ta.push_back({d.am[i], tile_code(TB_M, i)});
    for (int i = 0; i < d.tk; ++i) ta.push_back({d.ak[i], tile_code(TB_K, i)});
    for (int i = 0; i < d.tk; ++i) tb.push_back({d.bk[i], tile_code(TB_K, i)});
    for (int i = 0; i < d.tn; ++i) tb.push_back({d.bn[i], tile_code(TB_N, i)});
    for (int i = 0; i < d.tm; ++i) tc.push_back({d.cm[i], tile_code(TB_M, i)});
    for (int i = 0; i < d.tn; ++i) tc.push_back({d.cn[i], tile_code(TB_N, i)});
    tile_order(d.a_tile, ta);
    tile_order(d.b_tile, tb);
    tile_order(d.c_tile, tc);
    if (precision == MITNC_C64) {
      lds_row_swizzle(d.a_tile, d.tm + d.tk, TB_K, g.tm_bits, d.a_swz);
      lds_row_swizzle(d.b_tile, d.tk + d.tn, TB_K, g.tn_bits, d.b_swz);
    } else {
      lds_design_h(d, g);
    }
    // Split K over workgroups when there are too few output tiles to fill the
    // chip (Sec. V-B: partition along the common indices); keep at least 4 k
    // tiles per workgroup.
    // Workgroup target: the resident count of the TILE and TALL kernels (2
    // per CU, 512; measured on the 56-qubit share against 256 and 2048: the
    // split GEPDOT steps stream longer k ranges per workgroup with loads in
    // flight on every CU); SPLITK tiles are smaller and take 2^11.
    int tiles_bits = (d.mb - d.tm) + (d.nb - d.tn) + d.bb;
    int khigh = d.kb - d.tk;
    // Skinny split-K (complex64 SPLITK steps the skinny kernel takes): one
    // wave per split, 2^12 waves.
    const bool skinny = st.kclass == MITNC_K_SPLITK && precision == MITNC_C64 && d.mb + d.nb <= 4 &&
                        d.kb >= kSkinnyLaneBits + 2 && d.bb <= 16;
    int target_bits = P->opts.splitk_target_bits > 0 ? std::min(P->opts.splitk_target_bits, 16)
                      : st.kclass == MITNC_K_TILE                 ? MITNC_TILE_SPLIT_TARGET
                      : st.kclass == MITNC_K_TALL                 ? MITNC_TALL_SPLIT_TARGET
                      : skinny                                    ? 12
                                                                  : 11;
    int ks = 0;
    while (tiles_bits + ks < target_bits && ks + kSplitMinStageBits < khigh) ++ks;
    uint64_t c_elems = 1ull << (d.mb + d.nb + d.bb);
    while (ks > 0 && (c_elems << ks) * 8 > (256ull << 20)) --ks;
    d.ks_bits = ks;
    st.part_bytes = ks > 0 ? (c_elems << ks) * 8 : 0;
  }
  st.flops = 8.0 * std::ldexp(1.0, d.mb + d.nb + d.kb + d.bb);
  // Algorithmic HBM bytes: each operand read once, the output written once
  // (the last step of a slice reads and writes the complex128 sum instead).
  const double esz = precision == MITNC_C64 ? 8.0 : 4.0;
  st.bytes = esz * (std::ldexp(1.0, A.rank) + std::ldexp(1.0, B.rank)) +
             (st.root ? 32.0 : esz) * std::ldexp(1.0, O.rank);
}

// ---------------------------------------------------------------- fused sections
// A step can join a section when it contracts a large tensor (A) with a small
// matrix: no batch indices, K, N <= 64 and a padded B^T of at most
// kMaxSectionB entries.
static bool section_member_ok(const mitnc_plan* P, const PlanStep& st) {
  const StepDesc& d = st.d;
  if (st.root || d.bb != 0 || d.kb > 6 || d.nb > 6) return false;
  if (std::max(1 << d.kb, 4) * std::max(1 << d.nb, 16) > kMaxSectionB) return false;
  if ((d.kb > 2 ? d.kb - 2 : 0) + (d.nb > 4 ? d.nb - 4 : 0) > 4) return false;  // B fragments in registers
  if (P->nodes[st.a].rank < 14 || P->nodes[st.out].hoisted) return false;
  return true;
}

// Tile maps and step descriptors of a section over the chain `members`
// (members[j + 1] consumes the output of members[j] as its A).  The tile
// holds every label the section contracts that T already has, plus
// "passengers": the labels on T's four lowest address bits (coalescing) and
// more low labels until every step keeps at least 4 rows bits and the tile
// has at least 2^8 entries.  Inter-tile labels (Sec. IV: the ones that live
// longest) only select the tile.  Returns false when the tile would exceed
// 2^kMaxTileBits entries or LDS.
static bool build_section(const mitnc_plan* P, const std::vector<int>& members, int precision, PlanSection& sec) {
  const int L = (int)members.size();
  const PlanNode& Tin = P->nodes[P->steps[members[0]].a];
  const PlanNode& Tout = P->nodes[P->steps[members.back()].out];
  std::vector<std::vector<int64_t>> Kj(L), Nj(L);
  for (int j = 0; j < L; ++j) {
    const PlanStep& st = P->steps[members[j]];
    const PlanNode& A = P->nodes[st.a];
    const PlanNode& B = P->nodes[st.b];
    std::set<int64_t> sa(A.labels.begin(), A.labels.end());
    for (int64_t x : B.labels) (sa.count(x) ? Kj[j] : Nj[j]).push_back(x);
  }
  std::set<int64_t> tin(Tin.labels.begin(), Tin.labels.end()), tile;
  for (int j = 0; j < L; ++j)
    for (int64_t x : Kj[j])
      if (tin.count(x)) tile.insert(x);
  auto pos_in = [&](int64_t x) {
    for (size_t i = 0; i < Tin.labels.size(); ++i)
      if (Tin.labels[i] == x) return Tin.pos[i];
    return -1;
  };
  auto pos_out = [&](int64_t x) {
    for (size_t i = 0; i < Tout.labels.size(); ++i)
      if (Tout.labels[i] == x) return Tout.pos[i];
    return -1;
  };
  std::vector<std::pair<int, int64_t>> by_pos;  // T_in labels by address bit
  for (size_t i = 0; i < Tin.labels.size(); ++i) by_pos.push_back({Tin.pos[i], Tin.labels[i]});
  std::sort(by_pos.begin(), by_pos.end());
  for (auto& [p, x] : by_pos)
    if (p < 4) tile.insert(x);
  for (size_t i = 0; i < Tout.labels.size(); ++i)
    if (Tout.pos[i] < 4 && tin.count(Tout.labels[i])) tile.insert(Tout.labels[i]);
  int max_bits = 0, out_bits = 0;
  auto simulate = [&]() {
    bool ok = true;
    std::set<int64_t> cur = tile;
    max_bits = (int)cur.size();
    for (int j = 0; j < L; ++j) {
      if ((int)cur.size() - (int)Kj[j].size() < 4) ok = false;
      for (int64_t x : Kj[j]) cur.erase(x);
      for (int64_t x : Nj[j]) cur.insert(x);
      max_bits = std::max(max_bits, (int)cur.size());
    }
    out_bits = (int)cur.size();
    return ok && (int)tile.size() >= 8 && out_bits >= 8;
  };
  size_t next = 0;
  while (!simulate()) {
    while (next < by_pos.size() && tile.count(by_pos[next].second)) ++next;
    if (next >= by_pos.size()) return false;
    tile.insert(by_pos[next].second);
  }
  if (max_bits > kTileBitsTarget) return false;
  for (int64_t x : tin)
    if (!tile.count(x) && pos_out(x) < 0) return false;  // an inter-tile label must survive

  SectionDesc& sd = sec.sd;
  std::memset(&sd, 0, sizeof(sd));
  sd.n_steps = L;
  // One tile per workgroup iteration (tb_bits = 0).  The kernel can also
  // take 2^tb_bits tiles at a time (sharing each step's setup), but that
  // leaves fewer workgroups in flight and measured slower on MI355X.
  sd.stride_bits = max_bits;
  sd.tb_bits = 0;
  sd.tile_max = 1 << (max_bits + sd.tb_bits);
  // buffer 0: tile labels by A address bit; outer labels likewise
  std::vector<int64_t> lay;
  int no = 0;
  for (auto& [p, x] : by_pos) {
    if (tile.count(x)) {
      sd.p_in[lay.size()] = (uint8_t)p;
      lay.push_back(x);
    } else {
      sd.q_in[no] = (uint8_t)p;
      sd.q_out[no] = (uint8_t)pos_out(x);
      ++no;
    }
  }
  sd.t_in = (int)lay.size();
  sd.outer_bits = no;
  uint32_t b_off = 0;
  std::set<int64_t> cur(tile.begin(), tile.end());
  for (int j = 0; j < L; ++j) {
    const PlanStep& st = P->steps[members[j]];
    const PlanNode& B = P->nodes[st.b];
    std::map<int64_t, int> in_bit, out_bit, b_pos;
    for (size_t i = 0; i < lay.size(); ++i) in_bit[lay[i]] = (int)i;
    for (size_t i = 0; i < B.labels.size(); ++i) b_pos[B.labels[i]] = B.pos[i];
    std::set<int64_t> kset(Kj[j].begin(), Kj[j].end());
    std::vector<int64_t> M, Kv(Kj[j]);
    for (int64_t x : lay)
      if (!kset.count(x)) M.push_back(x);  // ascending input bit
    std::sort(Kv.begin(), Kv.end(), [&](int64_t u, int64_t v) { return in_bit[u] < in_bit[v]; });
    for (int64_t x : Kj[j]) cur.erase(x);
    for (int64_t x : Nj[j]) cur.insert(x);
    // output layout: the final one in C's address order; otherwise the next
    // step's four lane rows bits and two lane k bits lowest (conflict-free
    // LDS reads there), then the rest
    std::vector<int64_t> nlay;
    if (j == L - 1) {
      std::vector<std::pair<int, int64_t>> v;
      for (int64_t x : cur) v.push_back({pos_out(x), x});
      std::sort(v.begin(), v.end());
      for (auto& [p, x] : v) {
        sd.p_out[nlay.size()] = (uint8_t)p;
        nlay.push_back(x);
      }
    } else {
      // this step's lane rows bits, then its two lane n bits lowest: each
      // store instruction writes 64 consecutive entries; in a stem the next
      // step contracts the new bits, so its lane k bits are low as well
      std::vector<int64_t> first(M.begin(), M.begin() + 4);
      for (size_t i = 0; i < Nj[j].size() && i < 2; ++i) first.push_back(Nj[j][i]);
      std::set<int64_t> fs(first.begin(), first.end());
      nlay = first;
      for (int64_t x : Kj[j + 1])
        if (!fs.count(x) && cur.count(x)) {
          nlay.push_back(x);
          fs.insert(x);
        }
      for (int64_t x : cur)
        if (!fs.count(x)) nlay.push_back(x);
    }
    for (size_t i = 0; i < nlay.size(); ++i) out_bit[nlay[i]] = (int)i;
    std::vector<int64_t> Nv(Nj[j]);
    std::sort(Nv.begin(), Nv.end(), [&](int64_t u, int64_t v) { return out_bit[u] < out_bit[v]; });
    TileStep& ts = sd.st[j];
    ts.mb = (int)M.size();
    ts.kb = (int)Kv.size();
    ts.nb = (int)Nv.size();
    if (ts.mb > 16 || ts.kb > 8 || ts.nb > 8) return false;
    for (int i = 0; i < ts.mb; ++i) {
      ts.am[i] = (uint8_t)in_bit[M[i]];
      ts.cm[i] = (uint8_t)out_bit[M[i]];
    }
    for (int i = 0; i < ts.kb; ++i) {
      ts.ak[i] = (uint8_t)in_bit[Kv[i]];
      ts.bk[i] = (uint8_t)b_pos[Kv[i]];
    }
    for (int i = 0; i < ts.nb; ++i) {
      ts.cn[i] = (uint8_t)out_bit[Nv[i]];
      ts.bn[i] = (uint8_t)b_pos[Nv[i]];
    }
    ts.kpad = (uint32_t)std::max(1 << ts.kb, 4);
    ts.b_lds = b_off;
    b_off += (uint32_t)std::max(1 << ts.nb, 16) * ts.kpad;
    ts.out_scale = 1.f;
    ts.step_index = members[j];
    lay = nlay;
  }
  sd.t_out = (int)lay.size();
  sd.b_total = b_off;
  if ((2ull * sd.tile_max + sd.b_total) * 8 > kSectionMaxLds) return false;
  sec.steps = members;
  const double esz = precision == MITNC_C64 ? 8.0 : 4.0;
  sec.flops = 0;
  sec.bytes = esz * (std::ldexp(1.0, Tin.rank) + std::ldexp(1.0, Tout.rank));
  for (int m : members) {
    sec.flops += P->steps[m].flops;
    sec.bytes += esz * std::ldexp(1.0, P->nodes[P->steps[m].b].rank);
  }
  return true;
}

static void form_sections(mitnc_plan* P, int precision) {
  const int ns = (int)P->steps.size();
  std::vector<int> consumer(P->nodes.size(), -1);
  for (int s = 0; s < ns; ++s) consumer[P->steps[s].a] = consumer[P->steps[s].b] = s;
  for (int s = 0; s < ns; ++s) {
    if (P->step_section[s] >= 0 || !section_member_ok(P, P->steps[s])) continue;
    std::vector<int> mem{s};
    PlanSection best;
    bool have = false;
    while ((int)mem.size() < kMaxSectionSteps) {
      const PlanStep& last = P->steps[mem.back()];
      if (P->nodes[last.out].region != 2) break;  // a cached or final value must be stored
      const int u = consumer[last.out];
      if (u < 0) break;
      const PlanStep& su = P->steps[u];
      if (su.a != last.out || !section_member_ok(P, su) || P->nodes[su.out].lo != P->nodes[last.out].lo) break;
      mem.push_back(u);
      PlanSection cand;
      if (!build_section(P, mem, precision, cand)) break;
      best = cand;
      have = true;
    }
    if (!have) continue;
    const int id = (int)P->sections.size();
    for (int m : best.steps) P->step_section[m] = id;
    P->sections.push_back(best);
  }
}

// Operands a launch reads: a step's two, or a section's input and small
// tensors.  Returns false for steps that run inside a later launch.
static bool launch_operands(const mitnc_plan* P, int s, std::vector<int>& ops) {
  ops.clear();
  const int sec = P->step_section.empty() ? -1 : P->step_section[s];
  if (sec < 0) {
    ops = {P->steps[s].a, P->steps[s].b};
    return true;
  }
  const PlanSection& S = P->sections[sec];
  if (S.steps.back() != s) return false;
  ops.push_back(P->steps[S.steps[0]].a);
  for (int m : S.steps) ops.push_back(P->steps[m].b);
  return true;
}

// Replays the launch schedule of slices 0 .. n_slices-1 on the host with a
// map of which node value every workspace byte range holds, and fails if a
// step reads an operand whose bytes were overwritten since it was produced,
// or writes its output over one of its own operands.  It also checks that
// the value read is the one the reading slice needs: produced in a slice
// with the same bits of the operand's emask, and for a merge accumulator,
// summed over every pattern of its merged bits.
static void verify_memory_plan(const mitnc_plan* P, uint64_t n_slices) {
  struct Buf {
    uint64_t lo, hi;
    int node;
  };
  std::vector<Buf> held;
  auto range = [&](int node, uint64_t& lo, uint64_t& hi) {
    const PlanNode& nd = P->nodes[node];
    uint64_t base = nd.region == 0 ? 0 : nd.region == 1 ? P->off_persist : P->off_arena;
    lo = base + nd.offset;
    hi = lo + (nd.region == 0 ? P->leaf_data[nd.leaf_id].size() * 4 : (8ull << nd.full_rank));
  };
  auto overlaps = [](uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1) { return a0 < b1 && b0 < a1; };
  for (int i = 0; i < P->n_leaves; ++i) {
    uint64_t lo, hi;
    range(i, lo, hi);
    held.push_back({lo, hi, i});
  }
  const size_t nn = P->nodes.size();
  std::vector<uint64_t> vkey(nn, 0);     // emask bits (minus bmask) of the slice that produced the value
  std::vector<uint64_t> terms(nn, 0);    // accumulators: terms summed so far
  std::vector<uint64_t> last_pat(nn, 0); // accumulators: compressed merged bits of the last term
  SliceSchedule sched(nn);
  auto pattern_index = [](uint64_t s, uint64_t bm) {  // bits of s under bm, compressed
    uint64_t r = 0;
    int j = 0;
    for (; bm; bm &= bm - 1, ++j) r |= ((s >> __builtin_ctzll(bm)) & 1ull) << j;
    return r;
  };
  std::vector<int> ops;
  // A batched run executes level by level: every buffer its steps read or
  // write must be distinct from every other one of the run.
  for (size_t r = 0; r < P->fwd_runs.size(); ++r) {
    const mitnc_plan::FwdRun& R = P->fwd_runs[r];
    std::vector<int> nodes;
    for (int i = R.first_step; i <= R.last_step; ++i)
      if (P->fwd_run_of[i] == (int)r)
        for (int v : {P->steps[i].a, P->steps[i].b, P->steps[i].out})
          if (std::find(nodes.begin(), nodes.end(), v) == nodes.end()) nodes.push_back(v);
    for (size_t x = 0; x < nodes.size(); ++x)
      for (size_t y = x + 1; y < nodes.size(); ++y) {
        uint64_t a0, a1, b0, b1;
        range(nodes[x], a0, a1);
        range(nodes[y], b0, b1);
        if (overlaps(a0, a1, b0, b1)) fail(MITNC_INVALID_ARG, "internal: buffers of a batched run overlap");
      }
  }
  for (uint64_t s = 0; s < n_slices; ++s) {
    // the range prologue runs before the first slice, then its steps are skipped
    std::vector<std::pair<size_t, int>> seq;  // (step, mode) in launch order
    if (s == 0)
      for (int i : P->prologue_order) seq.push_back({(size_t)i, 1});
    for (size_t si = 0; si < P->steps.size(); ++si) {
      const PlanNode& O = P->nodes[P->steps[si].out];
      const int mode = sched.decide(P->steps[si].out, O.elig, O.emask, O.bmask, s);
      if (mode && P->fwd_run_of[si] < 0) seq.push_back({si, mode});
    }
    for (auto [si, mode] : seq) {
      const PlanStep& st = P->steps[si];
      const PlanNode& O = P->nodes[st.out];
      if (!launch_operands(P, (int)si, ops)) continue;  // runs with its section
      for (int node : ops) {
        uint64_t lo, hi;
        range(node, lo, hi);
        bool ok = false;
        for (auto& b : held)
          if (b.node == node && b.lo == lo && b.hi == hi) ok = true;
        if (!ok) fail(MITNC_INVALID_ARG, "internal: operand " + std::to_string(node) + " clobbered before use");
        const PlanNode& X = P->nodes[node];
        if (!X.leaf) {
          if (vkey[node] != (s & X.emask & ~X.bmask))
            fail(MITNC_INVALID_ARG, "internal: operand " + std::to_string(node) + " holds another slice's value");
          if (X.bmask && terms[node] != (1ull << __builtin_popcountll(X.bmask)))
            fail(MITNC_INVALID_ARG, "internal: merge accumulator " + std::to_string(node) + " read before complete");
        }
      }
      if (st.root) continue;
      uint64_t olo, ohi;
      range(st.out, olo, ohi);
      uint64_t wlo = olo, whi = ohi;  // bytes the step's kernel writes
      if (mode == 2) {
        wlo = P->off_arena + O.tmp_offset;
        whi = wlo + (8ull << O.full_rank);
        if (overlaps(wlo, whi, olo, ohi)) fail(MITNC_INVALID_ARG, "internal: merge term overlaps its accumulator");
      }
      for (int node : ops) {
        uint64_t lo, hi;
        range(node, lo, hi);
        if (overlaps(wlo, whi, lo, hi)) fail(MITNC_INVALID_ARG, "internal: step output overlaps an operand");
      }
      if (mode == 2) {
        bool ok = false;
        for (auto& b : held)
          if (b.node == (int)st.out && b.lo == olo && b.hi == ohi) ok = true;
        if (!ok) fail(MITNC_INVALID_ARG, "internal: merge accumulator " + std::to_string(st.out) + " clobbered");
        const uint64_t t = pattern_index(s, O.bmask);
        if (t <= last_pat[st.out] || vkey[st.out] != (s & O.emask & ~O.bmask))
          fail(MITNC_INVALID_ARG, "internal: merge term out of order");
        last_pat[st.out] = t;
        terms[st.out]++;
      } else {
        vkey[st.out] = s & O.emask & ~O.bmask;
        terms[st.out] = 1;  // pattern 0
        last_pat[st.out] = 0;
      }
      std::vector<Buf> keep;
      for (auto& b : held)
        if (!overlaps(b.lo, b.hi, wlo, whi) && !(mode == 1 && b.node == (int)st.out)) keep.push_back(b);
      if (mode == 1) keep.push_back({olo, ohi, (int)st.out});
      held.swap(keep);
    }
  }
}

void build_step_for(mitnc_plan* P, PlanStep& st, const std::vector<int64_t>& c_labels,
                    const std::vector<int64_t>* root_layout, int force_kernel, int precision) {
  build_step(P, st, c_labels, root_layout, force_kernel, precision);
}

// Reverse pass of the differentiation form: which nodes need an adjoint
// (a single-qubit gate leaf below them), where adjoints live, one adjoint
// contraction per (step, child needing it) in reverse step order, and the
// leaf-to-gradient table.
static void build_reverse(mitnc_plan* P, const mitnc_network* net, const mitnc_plan_opts& opts) {
  const int n = P->n_leaves;
  P->has_grad.assign(P->nodes.size(), 0);
  std::vector<int> gate_of_leaf(n, -1);
  int g1 = 0;
  for (int i = 0; i < n; ++i) {
    const Leaf& L = net->leaves[i];
    if (L.gate >= 0 && L.arity == 1) {
      P->has_grad[i] = 1;
      gate_of_leaf[i] = g1++;
    }
  }
  P->n_grad_gates = g1;
  for (auto& st : P->steps) P->has_grad[st.out] = P->has_grad[st.a] || P->has_grad[st.b];
  P->adj_offset.assign(P->nodes.size(), 0);
  uint64_t off = 0;
  for (size_t v = 0; v < P->nodes.size(); ++v) {
    if (!P->has_grad[v]) continue;
    P->adj_offset[v] = off;
    off = align_up(off + (8ull << P->nodes[v].rank), 256);
  }
  for (int si = (int)P->steps.size() - 1; si >= 0; --si) {
    const PlanStep& st = P->steps[si];
    if (!P->has_grad[st.out]) continue;
    for (int which = 0; which < 2; ++which) {
      const int target = which == 0 ? st.a : st.b;
      const int other = which == 0 ? st.b : st.a;
      if (!P->has_grad[target]) continue;
      mitnc_plan T;
      T.nodes.resize(3);
      const PlanNode& O = P->nodes[st.out];
      T.nodes[0].labels = O.labels;
      T.nodes[0].pos = O.pos;
      T.nodes[0].rank = O.rank;
      T.nodes[1].labels = P->nodes[other].labels;
      T.nodes[1].pos = P->nodes[other].pos;
      T.nodes[1].rank = P->nodes[other].rank;
      const std::vector<int64_t>& tl = P->nodes[target].labels;  // physical order, dense adjoint layout
      PlanStep rs;
      rs.a = 0;
      rs.b = 1;
      rs.out = 2;
      build_step(&T, rs, tl, &tl, opts.force_kernel, MITNC_C64);
      RevOp r;
      r.step = si;
      r.target = target;
      r.other = other;
      r.adj_is_a = rs.a == 0;
      r.kclass = rs.kclass;
      r.d = rs.d;
      r.part_bytes = rs.part_bytes;
      r.flops = rs.flops;
      P->rev_flops += rs.flops;
      P->rev.push_back(r);
    }
  }
  // Grouped reverse pass: deferral roots, chosen top-down (a node's parent
  // step comes later in the path), each with a term buffer after the
  // adjoints.  below[v]: reverse flops of the ops that read an adjoint in
  // v's subtree (the work a deferral at v would run once per run of slices).
  const int nn = (int)P->nodes.size();
  const int root = P->steps.back().out;
  std::vector<int> parent(nn, -1);
  for (auto& st : P->steps) parent[st.a] = parent[st.b] = st.out;
  std::vector<double> below(nn, 0.0);
  for (const RevOp& r : P->rev)
    for (int v = P->steps[r.step].out; v >= 0; v = parent[v]) below[v] += r.flops;
  P->defer_group.assign(nn, -1);
  P->adj_term_offset.assign(nn, 0);
  P->rev_groups.assign(1, mitnc_plan::RevGroup{});
  std::vector<int> group_of(nn, 0);  // innermost deferral root's group at or above each node
  auto lo_of = [&](int v) { return P->nodes[v].lo >= kLevelNever ? 64 : P->nodes[v].lo; };
  for (int si = (int)P->steps.size() - 1; si >= 0; --si) {
    const int v = P->steps[si].out;
    if (v == root) continue;
    group_of[v] = group_of[parent[v]];
    const int lo = lo_of(v), lp = lo_of(parent[v]);
    if (opts.reverse_defer < 0 || !P->has_grad[v] || lo <= lp) continue;
    // Saved: the subtree's reverse flops in all but one slice of each run
    // of 2^span; paid: the accumulation, 3 accesses of 8 bytes per adjoint
    // entry and slice.  The weight of 24 flops per entry follows measurement:
    // the reverse kernels of these subtrees are themselves HBM-bound (about
    // one flop per byte), so an accumulation costs about its bytes.
    const int span = std::min(lo, P->S);
    const double saved = below[v] * (1.0 - std::ldexp(1.0, -span));
    const double cost = 24.0 * std::ldexp(1.0, P->nodes[v].rank);
    if (opts.reverse_defer == 0 && (span == 0 || saved <= cost)) continue;
    const int g = (int)P->rev_groups.size();
    mitnc_plan::RevGroup G;
    G.root = v;
    G.lo = std::min(lo, 63);
    P->rev_groups.push_back(G);
    P->rev_groups[group_of[parent[v]]].children.push_back(g);
    group_of[v] = g;
    P->defer_group[v] = g;
    P->adj_term_offset[v] = off;
    off = align_up(off + (8ull << P->nodes[v].rank), 256);
  }
  P->adj_bytes = off;
  for (const RevOp& r : P->rev) P->rev_group_of.push_back(group_of[P->steps[r.step].out]);
  std::vector<std::pair<int, GradEntry>> tagged;  // (group of the op writing the leaf's adjoint, entry)
  for (int i = 0; i < n; ++i) {
    if (gate_of_leaf[i] < 0) continue;
    const PlanNode& nd = P->nodes[i];
    GradEntry e;
    std::memset(&e, 0, sizeof(e));
    e.adj_offset = P->adj_offset[i];  // made absolute once the workspace layout is known
    e.gate = gate_of_leaf[i];
    e.rank = nd.rank;
    for (int b = 0; b < nd.rank; ++b) e.full_pos[b] = (int8_t)nd.pos[b];
    e.n_sliced = (int8_t)nd.slice_bits.size();
    for (size_t j = 0; j < nd.slice_bits.size(); ++j) {
      e.slice_bit[j] = (int8_t)nd.slice_bits[j].first;
      e.slice_pos[j] = (int8_t)nd.slice_bits[j].second;
    }
    tagged.push_back({group_of[parent[i]], e});
  }
  std::stable_sort(tagged.begin(), tagged.end(),
                   [](const std::pair<int, GradEntry>& x, const std::pair<int, GradEntry>& y) { return x.first < y.first; });
  for (auto& [g, e] : tagged) {
    mitnc_plan::RevGroup& G = P->rev_groups[g];
    if (G.grad_count == 0) G.grad_first = (uint32_t)P->gtab.size();
    G.grad_count++;
    P->gtab.push_back(e);
  }
}

// Reverse pass by depth (needs the workspace offsets of nodes and adjoints):
// an op's level is one more than that of the op writing the adjoint it reads
// (0 for the root's).  SMALL ops of a level go into the batched-launch
// tables, one block-table entry per workgroup of 256 outputs.
// A reverse op goes into the batched SMALL launch when it is SMALL and
// within the class limits (a forced SMALL class on a larger shape runs alone).
static bool batched_small(const RevOp& r) {
  return r.kclass == MITNC_K_SMALL && small_bounded(r.d.mb, r.d.nb, r.d.kb, r.d.bb);
}

static void build_reverse_levels(mitnc_plan* P) {
  const int root = P->steps.back().out;
  std::vector<int> level_of(P->nodes.size(), -1);  // level of the op writing a node's adjoint
  for (size_t i = 0; i < P->rev.size(); ++i) {
    const RevOp& r = P->rev[i];
    const int in = P->steps[r.step].out;
    int lv = 0;
    if (in != root) {
      if (level_of[in] < 0) fail(MITNC_INVALID_ARG, "reverse schedule reads an adjoint before it is written");
      lv = level_of[in] + 1;
    }
    level_of[r.target] = lv;
    P->rev_level_of.push_back(lv);
    if ((int)P->rev_levels.size() <= lv) P->rev_levels.resize(lv + 1);
    if (!batched_small(r)) P->rev_levels[lv].big.push_back((int)i);
  }
  // Where an op writes: a deferral root's adjoint goes to its term buffer.
  auto write_off = [&](int target) {
    return P->off_adj + (P->defer_group[target] >= 0 ? P->adj_term_offset[target] : P->adj_offset[target]);
  };
  for (mitnc_plan::RevGroup& G : P->rev_groups) G.levels.assign(P->rev_levels.size(), mitnc_plan::RevLevel{});
  for (size_t gi = 0; gi < P->rev_groups.size(); ++gi)
    for (size_t lv = 0; lv < P->rev_levels.size(); ++lv) {
      mitnc_plan::RevLevel& L = P->rev_groups[gi].levels[lv];
      for (int i : P->rev_levels[lv].big)
        if (P->rev_group_of[i] == (int)gi) L.big.push_back(i);
      L.small_first = (uint32_t)P->rblock.size();
      for (size_t i = 0; i < P->rev.size(); ++i) {
        const RevOp& r = P->rev[i];
        if (!batched_small(r) || P->rev_level_of[i] != (int)lv || P->rev_group_of[i] != (int)gi) continue;
        SmallRevOp e;
        std::memset(&e, 0, sizeof(e));
        e.d = r.d;
        e.d.A = e.d.B = nullptr;
        e.d.C = nullptr;
        const uint64_t adj_in = P->off_adj + P->adj_offset[P->steps[r.step].out];
        const PlanNode& o = P->nodes[r.other];
        uint64_t other = o.offset;
        if (o.region == 1) other += P->off_persist;
        else if (o.region == 2) other += P->off_arena;
        else if (o.region != 0) fail(MITNC_INVALID_ARG, "reverse operand outside the workspace");
        e.a_off = r.adj_is_a ? adj_in : other;
        e.b_off = r.adj_is_a ? other : adj_in;
        e.c_off = write_off(r.target);
        if (o.region == 0 && !o.slice_bits.empty()) {
          if (o.slice_bits.size() > 8) fail(MITNC_UNSUPPORTED, "leaf with more than 8 sliced indices");
          e.sl_which = r.adj_is_a ? 2 : 1;
          e.sl_n = (int8_t)o.slice_bits.size();
          for (size_t j = 0; j < o.slice_bits.size(); ++j) {
            e.sl_bit[j] = (int8_t)o.slice_bits[j].first;
            e.sl_pos[j] = (int8_t)o.slice_bits[j].second;
          }
        }
        const uint64_t c_elems = 1ull << (r.d.mb + r.d.nb + r.d.bb);
        e.block0 = (uint32_t)P->rblock.size();
        const uint32_t idx = (uint32_t)P->rtab.size();
        for (uint64_t b = 0; b < (c_elems + 255) / 256; ++b) P->rblock.push_back(idx);
        P->rtab.push_back(e);
      }
      L.small_blocks = (uint32_t)P->rblock.size() - L.small_first;
    }
}

// Tables of the batched forward SMALL runs (workspace offsets are known):
// per run and level, one table entry per step and one block-table entry per
// workgroup of 256 outputs; the FP16/BF16 plan's own geometry in ftab, the
// complex64 geometry of its calibration slices in ftab64.
static void build_forward_batches(mitnc_plan* P) {
  const bool half = P->opts.precision != MITNC_C64;
  auto node_off = [&](int node, bool h) -> uint64_t {
    const PlanNode& nd = P->nodes[node];
    if (nd.region == 0) return h ? P->off_leaf_half + nd.offset / 2 : nd.offset;
    if (nd.region == 1) return P->off_persist + nd.offset;
    if (nd.region == 2) return P->off_arena + nd.offset;
    fail(MITNC_INVALID_ARG, "internal: batched step output outside the workspace");
  };
  const std::vector<int>& level = P->fwd_levels_tmp;
  for (size_t r = 0; r < P->fwd_runs.size(); ++r) {
    mitnc_plan::FwdRun& R = P->fwd_runs[r];
    int nlev = 0;
    for (int i = R.first_step; i <= R.last_step; ++i)
      if (P->fwd_run_of[i] == (int)r) nlev = std::max(nlev, level[P->steps[i].out] + 1);
    for (int l = 0; l < nlev; ++l)
      for (int i = R.first_step; i <= R.last_step; ++i)
        if (P->fwd_run_of[i] == (int)r && level[P->steps[i].out] == l) P->prologue_order.push_back(i);
    for (int pass = 0; pass < (half ? 2 : 1); ++pass) {
      const bool h = half && pass == 0;  // pass 0: the plan's precision; pass 1: complex64 calibration
      std::vector<SmallFwdOp>& tab = pass == 0 ? P->ftab : P->ftab64;
      std::vector<uint32_t>& blk = pass == 0 ? P->fblock : P->fblock64;
      std::vector<mitnc_plan::FwdBatch>& lv = pass == 0 ? R.levels : R.levels64;
      lv.assign(nlev, mitnc_plan::FwdBatch{});
      for (int l = 0; l < nlev; ++l) {
        lv[l].first = (uint32_t)blk.size();
        for (int i = R.first_step; i <= R.last_step; ++i) {
          const PlanStep& st = P->steps[i];
          if (P->fwd_run_of[i] != (int)r || level[st.out] != l) continue;
          if (st.kclass != MITNC_K_SMALL || !small_bounded(st.d.mb, st.d.nb, st.d.kb, st.d.bb)) {
            if (pass == 0) lv[l].big.push_back(i);  // launched on its own, in its level
            continue;
          }
          SmallFwdOp e;
          std::memset(&e, 0, sizeof(e));
          e.d = pass == 0 ? st.d : st.d64;
          for (auto& [b, pos] : P->nodes[st.a].slice_bits) {
            e.a_bit[e.na] = (int8_t)b;
            e.a_pos[e.na++] = (int8_t)pos;
          }
          for (auto& [b, pos] : P->nodes[st.b].slice_bits) {
            e.b_bit[e.nb] = (int8_t)b;
            e.b_pos[e.nb++] = (int8_t)pos;
          }
          e.d.A = e.d.B = nullptr;
          e.d.C = nullptr;
          e.d.acc = nullptr;
          e.d.part = nullptr;
          e.d.stats = nullptr;
          e.d.step_index = i;
          e.d.mode = EPI_STORE;
          if (!h) e.d.out_scale = 1.f;
          e.a_off = node_off(st.a, h);
          e.b_off = node_off(st.b, h);
          e.c_off = node_off(st.out, h);
          const uint64_t c_elems = 1ull << (e.d.mb + e.d.nb + e.d.bb);
          e.block0 = (uint32_t)blk.size();
          const uint32_t idx = (uint32_t)tab.size();
          for (uint64_t b = 0; b < (c_elems + 255) / 256; ++b) blk.push_back(idx);
          tab.push_back(e);
          if (pass == 0) P->ftab_step.push_back(i);
          lv[l].flops += st.flops;
          lv[l].bytes += st.bytes;
        }
        lv[l].blocks = (uint32_t)blk.size() - lv[l].first;
      }
    }
  }
  std::vector<int>().swap(P->fwd_levels_tmp);
}

mitnc_plan* build_plan(const mitnc_network* net, const mitnc_plan_opts& opts) {
  if (!net->output_set) fail(MITNC_INVALID_ARG, "output not set");
  int n = (int)net->leaves.size();
  if (n < 2) fail(MITNC_UNSUPPORTED, "network needs at least two tensors");
  if (net->path.empty()) fail(MITNC_PATH_INVALID, "no path set");
  validate_path(n, net->path);
  if (opts.precision != MITNC_C64 && opts.precision != MITNC_CF16 && opts.precision != MITNC_CBF16)
    fail(MITNC_INVALID_ARG, "unknown precision");
  if (opts.merge_bits < 0 || opts.merge_bits > 12) fail(MITNC_INVALID_ARG, "merge_bits out of range (0..12)");
  if (opts.prologue_bits < 0 || opts.prologue_bits > 62) fail(MITNC_INVALID_ARG, "prologue_bits out of range (0..62)");
  auto P = std::make_unique<mitnc_plan>();
  P->opts = opts;
  P->n_leaves = n;
  P->S = (int)net->sliced.size();
  int S = P->S;
  if (S > 62) fail(MITNC_UNSUPPORTED, "too many sliced indices");
  std::map<int64_t, int> slice_bit;  // label -> slice-id bit (last listed = bit 0)
  for (int j = 0; j < S; ++j) slice_bit[net->sliced[j]] = S - 1 - j;

  SymNet sn = make_symnet(net->leaves, net->output_lsb);
  std::vector<char> slm(sn.n_labels, 0);
  for (auto x : net->sliced) {
    auto it = sn.dense.find(x);
    if (it == sn.dense.end() || !sn.closed[it->second]) fail(MITNC_INVALID_ARG, "sliced label is not a closed edge");
    slm[it->second] = 1;
  }
  auto sym = sym_run(sn, net->path, slm);
  P->max_log2 = sym_max_bits(sn, sym, slm);

  // Hoisting (same aim as the reuse of Sec. III-B, applied to sliced indices):
  // a small subtree that depends on sliced indices would be recomputed for
  // every slice, one tiny launch per step.  Instead it is contracted once
  // with its sliced indices kept as ordinary (batch) indices, and each slice
  // reads the sub-tensor of its index values, as it does for a sliced leaf.
  // Chosen: maximal non-root subtrees whose every intermediate, sliced bits
  // included, has at most 2^kHoistBits entries.
  constexpr int kHoistBits = 14;
  const int nsteps = (int)net->path.size();
  std::vector<uint64_t> smask(n + nsteps, 0);  // slice-id bits below each node
  for (int i = 0; i < n; ++i)
    for (int64_t x : net->leaves[i].labels) {
      auto it = slice_bit.find(x);
      if (it != slice_bit.end()) smask[i] |= 1ull << it->second;
    }
  std::vector<char> fits(n + nsteps, 1);  // whole subtree within the size cap
  for (int s = 0; s < nsteps; ++s) {
    const int a = net->path[s].first, b = net->path[s].second, o = n + s;
    smask[o] = smask[a] | smask[b];
    const int bits = (int)sym[s].c.size() + __builtin_popcountll(smask[o]);
    fits[o] = fits[a] && fits[b] && bits <= kHoistBits;
  }
  std::vector<char> in_hoist(n + nsteps, 0);
  std::vector<int> hoist_root(n + nsteps, 0);
  if (opts.reuse && !opts.differentiable && !opts.no_hoist) {
    std::vector<int> parent(n + nsteps, -1);
    for (int s = 0; s < nsteps; ++s) parent[net->path[s].first] = parent[net->path[s].second] = n + s;
    for (int s = 0; s < nsteps - 1; ++s) {
      const int o = n + s;
      const int p = parent[o];
      const bool parent_hoistable = p >= 0 && p != n + nsteps - 1 && fits[p] && smask[p] != 0;
      if (fits[o] && smask[o] != 0 && !parent_hoistable) hoist_root[o] = 1;
    }
    // mark subtrees (children come before parents in path order)
    for (int s = nsteps - 1; s >= 0; --s) {
      const int o = n + s;
      if (hoist_root[o]) in_hoist[o] = 1;
      if (in_hoist[o]) in_hoist[net->path[s].first] = in_hoist[net->path[s].second] = 1;
    }
  }
  std::map<int, int64_t> label_of_bit;
  for (auto& [x, b] : slice_bit) label_of_bit[b] = x;

  // Leaves.
  P->nodes.resize(n + net->path.size());
  uint64_t off = 0;
  for (int i = 0; i < n; ++i) {
    const Leaf& L = net->leaves[i];
    PlanNode& nd = P->nodes[i];
    nd.leaf = true;
    nd.leaf_id = i;
    nd.region = 0;
    for (size_t b = 0; b < L.labels.size(); ++b) {
      auto it = slice_bit.find(L.labels[b]);
      if (it != slice_bit.end()) nd.dmask |= 1ull << it->second;
      if (it != slice_bit.end() && !in_hoist[i]) {
        nd.slice_bits.push_back({it->second, (int)b});
      } else {
        nd.labels.push_back(L.labels[b]);
        nd.pos.push_back((int)b);
      }
    }
    nd.rank = (int)nd.labels.size();
    nd.full_rank = (int)L.labels.size();
    nd.hoisted = in_hoist[i];
    std::vector<float> h(L.data.size() * 2);
    for (size_t e = 0; e < L.data.size(); ++e) {
      h[2 * e] = (float)L.data[e].real();
      h[2 * e + 1] = (float)L.data[e].imag();
    }
    if (opts.precision != MITNC_C64) {
      double mx = 0;
      for (auto& z : L.data) mx = std::max(mx, std::max(std::fabs(z.real()), std::fabs(z.imag())));
      nd.exp = mantissa_exponent(mx);
      std::vector<uint32_t> w(L.data.size());
      for (size_t e = 0; e < L.data.size(); ++e) {
        float re = (float)std::ldexp(L.data[e].real(), -nd.exp), im = (float)std::ldexp(L.data[e].imag(), -nd.exp);
        w[e] = opts.precision == MITNC_CF16 ? (host_f16(re) | (host_f16(im) << 16))
                                            : (host_bf16(re) | (host_bf16(im) << 16));
      }
      P->leaf_half.push_back(std::move(w));
    }
    P->leaf_data.push_back(std::move(h));
    P->leaf_is_1q.push_back(L.gate >= 0 && L.arity == 1);
    nd.offset = off;
    off = align_up(off + L.data.size() * 8, 256);
  }
  P->leaf_bytes = off;

  // Steps: layouts and descriptors in path order.
  P->steps.resize(net->path.size());
  for (size_t s = 0; s < net->path.size(); ++s) {
    PlanStep& st = P->steps[s];
    st.a = net->path[s].first;
    st.b = net->path[s].second;
    st.out = n + (int)s;
    st.root = (s + 1 == net->path.size());
    P->nodes[st.a].parent = st.out;
    P->nodes[st.b].parent = st.out;
    std::vector<int64_t> cset;
    for (int x : sym[s].c) cset.push_back(sn.label_id[x]);
    const bool hz = in_hoist[st.out];
    if (hz)  // sliced indices below stay open
      for (int b = 0; b < S; ++b)
        if (smask[st.out] >> b & 1) cset.push_back(label_of_bit[b]);
    if (opts.precision != MITNC_C64) {
      // Calibration slices run in complex64, whose tiles differ: keep both.
      build_step(P.get(), st, cset, st.root ? &net->output_lsb : nullptr, opts.force_kernel, MITNC_C64);
      st.d64 = st.d;
      const uint64_t pb64 = st.part_bytes;
      build_step(P.get(), st, cset, st.root ? &net->output_lsb : nullptr, opts.force_kernel, opts.precision);
      st.part_bytes = std::max(st.part_bytes, pb64);
    } else {
      build_step(P.get(), st, cset, st.root ? &net->output_lsb : nullptr, opts.force_kernel, opts.precision);
    }
    PlanNode& O = P->nodes[st.out];
    O.dmask = P->nodes[st.a].dmask | P->nodes[st.b].dmask;
    O.hoisted = hz;
    // Work of the step inside one slice: a hoisted step covers 2^(sliced
    // indices below it) slices at once.
    const double per = hz ? std::ldexp(1.0, -__builtin_popcountll(smask[st.out])) : 1.0;
    st.flops_slice = st.flops * per;
    st.bytes_slice = st.bytes * per;
    if (hoist_root[st.out]) {
      // Seen from its consumer the hoisted result is sliced like a leaf.
      std::vector<int64_t> lab;
      std::vector<int> pos;
      for (size_t i = 0; i < O.labels.size(); ++i) {
        auto it = slice_bit.find(O.labels[i]);
        if (it != slice_bit.end()) {
          O.slice_bits.push_back({it->second, O.pos[i]});
        } else {
          lab.push_back(O.labels[i]);
          pos.push_back(O.pos[i]);
        }
      }
      O.labels = lab;
      O.pos = pos;
      O.rank = (int)lab.size();
    }
  }
  // Recompute rule (SliceSchedule): without merges a node runs when one of
  // its slice-id bits changes (pre-lifetime reuse); every node runs in
  // every slice without reuse; hoisted nodes run once per range.  With
  // merge_bits, the post-lifetime merge of merge_sets on top.
  const int nn = (int)P->nodes.size();
  for (int u = 0; u < nn; ++u) {
    PlanNode& nd = P->nodes[u];
    nd.emask = !opts.reuse ? ~0ull : (nd.hoisted ? 0 : nd.dmask);
    nd.elig = nd.bmask = 0;
  }
  if (opts.merge_bits > 0 && opts.reuse) {
    std::vector<std::pair<int, int>> kids(nn, {-1, -1});
    std::vector<uint64_t> dm(nn);
    std::vector<char> hz(nn);
    for (int u = 0; u < nn; ++u) {
      dm[u] = P->nodes[u].dmask;
      hz[u] = P->nodes[u].hoisted;
    }
    for (auto& st : P->steps) kids[st.out] = {st.a, st.b};
    const MergeSets m = merge_sets(kids, dm, hz, std::min(opts.merge_bits, S));
    for (int u = n; u < nn; ++u) {
      P->nodes[u].elig = m.elig[u];
      P->nodes[u].emask = m.emask[u];
      P->nodes[u].bmask = P->steps[u - n].root ? 0 : m.bmask[u];
    }
    P->merged = m.merged;
    P->merge_align_bits = m.align_bits;
  }
  auto set_lo = [&](PlanNode& nd) { nd.lo = nd.emask ? __builtin_ctzll(nd.emask) : kLevelNever; };
  for (auto& nd : P->nodes) set_lo(nd);
  // Region choice: a node recomputed less often than its parent (both run
  // in the same slices otherwise) is kept, and so is a merge accumulator.
  auto assign_regions = [&]() {
    uint64_t pb = 0;
    for (size_t s = 0; s < P->steps.size(); ++s) {
      PlanNode& O = P->nodes[P->steps[s].out];
      if (P->steps[s].root) {
        O.region = 3;
        continue;
      }
      int lp = P->nodes[O.parent].lo;
      O.region = (O.lo > lp || O.bmask) ? 1 : 2;
      if (O.region == 1) pb += std::ldexp(8.0, O.full_rank);
    }
    return pb;
  };
  uint64_t pbytes = assign_regions();
  if (opts.cache_budget_bytes > 0) {
    // Demotion: the largest kept node runs whenever its parent does.
    while (pbytes > opts.cache_budget_bytes) {
      int best = -1;
      for (size_t s = 0; s < P->steps.size(); ++s) {
        PlanNode& O = P->nodes[P->steps[s].out];
        if (O.region == 1 && !O.hoisted && !O.bmask && O.lo > P->nodes[O.parent].lo &&
            (best < 0 || O.rank > P->nodes[best].rank))
          best = P->steps[s].out;
      }
      if (best < 0) break;
      P->nodes[best].emask |= P->nodes[P->nodes[best].parent].emask;
      set_lo(P->nodes[best]);
      pbytes = assign_regions();
    }
  }
  if (P->merged && (opts.differentiable || opts.fuse_sections))
    fail(MITNC_UNSUPPORTED, "post-lifetime merge is not combined with differentiable plans or fused sections");
  // Differentiable plans keep every node (the reverse pass reads them all).
  if (opts.differentiable) {
    if (opts.precision != MITNC_C64) fail(MITNC_UNSUPPORTED, "differentiable plans are complex64 only");
    for (auto& st : P->steps)
      if (!st.root) P->nodes[st.out].region = 1;
  }
  // Fused stem sections (Sec. IV): decided once regions are known (an
  // intermediate inside a section must be transient).
  P->step_section.assign(P->steps.size(), -1);
  if (opts.fuse_sections && opts.force_kernel < 0 && !opts.differentiable) form_sections(P.get(), opts.precision);
  // The range prologue: forward steps a slice range computes once (their
  // sliced indices, if any, all at slice-id bits >= prologue_bits, which a
  // range inside one aligned block of 2^prologue_bits slices keeps fixed;
  // hoisted ones; also those the merge schedule would only run at a later
  // slice of the range), run before the range's first slice level by level
  // (a level's steps read leaves and outputs of earlier levels); a level's
  // SMALL steps go out in one batched launch.
  P->fwd_run_of.assign(P->steps.size(), -1);
  const int pw = opts.prologue_bits;
  const uint64_t low = pw > 0 ? (1ull << pw) - 1 : ~0ull;  // bits that may vary inside a range
  auto fixed_bits = [&](const PlanNode& nd) {
    for (auto& [b, pos] : nd.slice_bits)
      if (pw == 0 || b < pw || (int)nd.slice_bits.size() > 16) return false;
    return true;
  };
  if (!opts.differentiable) {
    std::vector<int> level(P->nodes.size(), -1);
    std::vector<int> chosen;
    for (size_t i = 0; i < P->steps.size(); ++i) {
      const PlanStep& st = P->steps[i];
      const PlanNode& O = P->nodes[st.out];
      if (st.root || P->step_section[i] >= 0) continue;
      if ((O.emask & low) || O.bmask) continue;
      if (!fixed_bits(P->nodes[st.a]) || !fixed_bits(P->nodes[st.b])) continue;
      // operands: leaves, or outputs of prologue steps (anything else is
      // computed after the prologue)
      if ((st.a >= n && level[st.a] < 0) || (st.b >= n && level[st.b] < 0)) continue;
      int lv = 0;
      for (int o : {st.a, st.b})
        if (level[o] >= 0) lv = std::max(lv, level[o] + 1);
      level[st.out] = lv;
      chosen.push_back((int)i);
    }
    if (chosen.size() >= 2) {
      for (int i : chosen) {
        P->fwd_run_of[i] = 0;
        // A step the schedule would run later (waiting for merged bits) is
        // read at that later slice: its output is kept.
        if (P->nodes[P->steps[i].out].elig) P->nodes[P->steps[i].out].region = 1;
      }
      mitnc_plan::FwdRun R;
      R.first_step = chosen.front();
      R.last_step = chosen.back();
      P->fwd_runs.push_back(R);
    }
    P->fwd_levels_tmp.swap(level);
  }
  // Memory: persistent slots, then a transient arena with first-fit reuse.
  uint64_t poff = 0;
  for (auto& st : P->steps) {
    PlanNode& O = P->nodes[st.out];
    if (O.region == 1) {
      O.offset = poff;
      poff = align_up(poff + (8ull << O.full_rank), 256);
    }
  }
  P->persist_bytes = poff;
  std::vector<std::pair<uint64_t, uint64_t>> live;  // (offset, size) of live transient buffers
  std::vector<int> live_node;
  std::vector<int> pending;  // operands to release once the prologue has run
  uint64_t arena = 0;
  std::vector<int> ops;
  // The prologue's steps come first (their outputs live until their
  // consumers, operands until the prologue ends); then the others in order.
  std::vector<size_t> order;
  for (size_t s = 0; s < P->steps.size(); ++s)
    if (P->fwd_run_of[s] >= 0) order.push_back(s);
  const size_t n_pro = order.size();
  for (size_t s = 0; s < P->steps.size(); ++s)
    if (P->fwd_run_of[s] < 0) order.push_back(s);
  for (size_t oi = 0; oi < order.size(); ++oi) {
    const size_t s = order[oi];
    PlanStep& st = P->steps[s];
    // A section's steps run at its last step: earlier ones store nothing and
    // release nothing (the section's input and small tensors stay live).
    if (!launch_operands(P.get(), (int)s, ops)) continue;
    // The output is placed while the operands are still live (a kernel must
    // never write over its own inputs); the operands are released afterwards.
    PlanNode& O = P->nodes[st.out];
    auto place = [&](uint64_t sz) {
      std::vector<std::pair<uint64_t, uint64_t>> sorted = live;
      std::sort(sorted.begin(), sorted.end());
      uint64_t cand = 0;
      for (auto& [o, z] : sorted) {
        if (cand + sz <= o) break;
        cand = std::max(cand, o + z);
      }
      arena = std::max(arena, cand + sz);
      return cand;
    };
    if (O.region == 2) {
      uint64_t sz = align_up(8ull << O.full_rank, 256);
      O.offset = place(sz);
      live.push_back({O.offset, sz});
      live_node.push_back(st.out);
    }
    // A merge accumulator's later terms are computed into a transient buffer
    // and then added; the buffer is free again after the step.
    if (O.bmask) O.tmp_offset = place(align_up(8ull << O.full_rank, 256));
    // Operands of the prologue's steps stay allocated until it ends (its
    // steps run level by level, not in step order).
    for (int op : ops) pending.push_back(op);
    if (oi + 1 < n_pro) continue;
    for (int op : pending) {
      for (size_t i = 0; i < live_node.size(); ++i)
        if (live_node[i] == op) {
          live.erase(live.begin() + i);
          live_node.erase(live_node.begin() + i);
          break;
        }
    }
    pending.clear();
  }
  P->arena_bytes = arena;
  uint64_t part = 0;
  for (auto& st : P->steps) part = std::max(part, st.part_bytes);
  P->part_bytes = align_up(part, 256);
  P->result_elems = 1ull << net->output_lsb.size();
  if (opts.differentiable) build_reverse(P.get(), net, opts);
  for (auto& r : P->rev) P->part_bytes = std::max(P->part_bytes, align_up(r.part_bytes, 256));
  const bool half = opts.precision != MITNC_C64;
  // The 16-bit leaf region mirrors the complex64 one at half the offsets;
  // intermediates keep complex64 sizing so a calibration slice can run in
  // complex64 inside the same workspace.
  P->off_leaf_half = align_up(P->leaf_bytes, 256);
  P->off_persist = align_up(P->off_leaf_half + (half ? P->leaf_bytes / 2 : 0), 256);
  P->off_arena = align_up(P->off_persist + P->persist_bytes, 256);
  P->off_part = align_up(P->off_arena + P->arena_bytes, 256);
  P->off_stats = align_up(P->off_part + P->part_bytes, 256);
  P->off_calib = align_up(P->off_stats + 4 * P->steps.size(), 256);
  P->off_adj = align_up(P->off_calib + (half ? 16 * P->result_elems : 0), 256);
  P->off_gtab = align_up(P->off_adj + P->adj_bytes, 256);
  for (auto& g : P->gtab) g.adj_offset += P->off_adj;
  if (opts.differentiable) build_reverse_levels(P.get());
  P->off_rtab = align_up(P->off_gtab + sizeof(GradEntry) * P->gtab.size(), 256);
  P->off_rblock = align_up(P->off_rtab + sizeof(SmallRevOp) * P->rtab.size(), 256);
  build_forward_batches(P.get());
  P->off_ftab = align_up(P->off_rblock + sizeof(uint32_t) * P->rblock.size(), 256);
  P->off_fblock = align_up(P->off_ftab + sizeof(SmallFwdOp) * P->ftab.size(), 256);
  P->off_ftab64 = align_up(P->off_fblock + sizeof(uint32_t) * P->fblock.size(), 256);
  P->off_fblock64 = align_up(P->off_ftab64 + sizeof(SmallFwdOp) * P->ftab64.size(), 256);
  P->ws_bytes = align_up(P->off_fblock64 + sizeof(uint32_t) * P->fblock64.size(), 256);
  P->calibrated = !half;
  uint64_t n_check = std::min<uint64_t>(1ull << std::min(P->S, 62), 1ull << std::max(6, P->merge_align_bits + 1));
  if (opts.prologue_bits > 0) n_check = std::min<uint64_t>(n_check, 1ull << opts.prologue_bits);
  verify_memory_plan(P.get(), n_check);
  return P.release();
}

}  // namespace mitnc
