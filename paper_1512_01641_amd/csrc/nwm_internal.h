// Internal declarations shared by the HIP kernels and the C ABI of libnwmine.
// gfx950 (CDNA4) only: wave64, MFMA, 160 KiB LDS per CU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nwm {

// ---- tiling of the similarity contraction --------------------------------
// One wave computes a TM x TN tile of S for one document pair; the K
// dimension (the vocabulary, or the tile's target-side vocabulary) is walked
// in chunks of KC words.
constexpr int TM = 64;
constexpr int TN = 64;
constexpr int KC = 32;
// LDS row pitch (elements) of the dense operand tiles.
constexpr int PITCH_BF16 = KC + 8;   // 80 B rows: conflict-free ds_read_b128
constexpr int PITCH_F32 = KC + 4;    // 144 B rows

// List entries of one K chunk held in registers per lane by the contraction
// over the whole vocabulary (A: 128 entries, B: 128).  Every chunk load reads
// that many entries from the chunk start, so the lists carry that much slack
// at their end.
constexpr int REG_A = 2;
constexpr int REG_B = 2;
// The compacted contraction (K restricted to the column tile's words) holds
// up to 64 * CREG_A entries of a compacted chunk's A range in registers, for
// three chunks at a time.
constexpr int CREG_A = 5;
constexpr int CREG_B = 2;
constexpr int LIST_SLACK_A = 64 * (CREG_A > REG_A ? CREG_A : REG_A);
constexpr int LIST_SLACK_B = 64 * (CREG_B > REG_B ? CREG_B : REG_B);

// ---- dictionary-row merge ---------------------------------------------------
constexpr int MERGE_SLOTS = 1024;     // bound on tokens x max_deg per source sentence
constexpr int MAX_V = 32768;          // vocabulary bound (LDS tables of V / 32 words per tile)
constexpr int MAX_DEG = 64;           // dictionary entries per word

// ---- NW wavefront -----------------------------------------------------------
constexpr int BND_PAD = 192;          // slack slots after each published boundary row
// slots per published boundary row: even, so every row starts 16-byte aligned
__host__ __device__ inline int64_t bnd_stride(int m) { return ((int64_t)m + BND_PAD + 1) & ~(int64_t)1; }
constexpr int MAX_M = 1 << 22;           // target sentences per pair (a 64-row strip of S stays below 1 GiB)
constexpr int32_t ITEM_HOT = 1 << 30;   // DP item flag: strip of a critical-chain pair
// DP task slot flags (the LDS-ring fill runs four strips per workgroup): the
// strip's top boundary comes from the slot before it through LDS, and its
// last row goes to the slot after it through LDS
constexpr int32_t ITEM_LINK_IN = 1 << 29;
constexpr int32_t ITEM_LINK_OUT = 1 << 28;
constexpr int32_t ITEM_STRIP = ITEM_LINK_OUT - 1;   // the strip index bits
constexpr int FILL_SLOTS = 4;                        // strips (waves) per task of the LDS-ring fill
// Steps a strip trails the strip above it (the 63-step skew of a 64-row
// strip, a 16-step publish chunk, the two-chunk window prefetch and the
// hand-off's memory round trip): the queue order spaces a pair's strips by it.
constexpr int STRIP_LAG = 128;
// Pairs whose DP dependency chain is at least this percent of the longest are
// the "long" pairs: prepared, scored and aligned ahead of the others.
constexpr int LONG_CHAIN_PERCENT = 10;
// Of those, the pairs whose chain is at least this percent of the longest are
// the "top" pairs: scored first, their DP started as soon as their own tiles
// are scored.
constexpr int TOP_CHAIN_PERCENT = 60;

// Direction codes of the traceback.
constexpr int DIR_DIAG = 0, DIR_UP = 1, DIR_LEFT = 2;

// Traceback bits: per pair, per 64-row strip, per 64-step block, per lane
// (row) one uint4 = four 32-bit words of 16 steps x 2 bits (first step in the
// high bits).  ceil((m + 63) / 64) blocks per strip, 1 KiB per block.

// Everything the contraction needs about one tile, in one 64-byte record.
struct GtMeta {
  int32_t rt, ct, pair, m;
  int32_t row0, rows, col0, cols;
  int64_t s_first, t_first;   // first source / target sentence of the tile
  int64_t s_off;              // element offset of the pair's S block
  int64_t pad;
};

// A row tile (source side) or column tile (target side) in one 16-byte
// record: its first sentence (batch-wide index), sentence count and pair.
struct TileMeta {
  int64_t first;
  int32_t count, pair;
};

// Device-resident per-pair metadata of a plan.
struct PlanDev {
  int B;
  int V;
  int max_deg;
  int nch;                 // ceil(V / KC)
  const int32_t *n, *m;    // [B]
  const int64_t *sfirst;   // [B+1] first source sentence of each pair
  const int64_t *tfirst;   // [B+1]
  const int64_t *s_off;    // [B+1] element offset of S blocks
  const int64_t *p_off;    // [B+1] pair offset of path / kept lists
  const int64_t *tb_off;   // [B+1] byte offset of traceback bits
  int64_t path_base;       // byte offset of the path area inside tb
  // row tiles (source side) and column tiles (target side)
  int n_rt, n_ct;
  const int32_t *rt_pair, *rt_row0, *rt_rows;
  const int32_t *ct_pair, *ct_col0, *ct_cols;
  const TileMeta *rt_meta, *ct_meta;
  // contraction tiles: (row tile, column tile)
  int n_gt;
  const int32_t *gt_rt, *gt_ct;
  const GtMeta *gt_meta;
  // DP order (longest first) and DP work items (pair, strip) in queue order
  const int32_t *dp_order;
  const int64_t *sent_ids;   // [sum n] source sentences, long pairs' first
  int n_items;
  const int32_t *it_pair, *it_strip;
  // the same strips as tasks of FILL_SLOTS slots (pair -1: an empty slot)
  int n_tasks;
  const int32_t *tk_pair, *tk_slot;
  const int64_t *bnd_off;   // [B+1] offset of a pair's published boundary rows (uint64 units)
};

// Workspace layout (byte offsets into the caller's ws).
struct WsLayout {
  size_t a_merged;   // uint2 {u, f32 bits} [src_tokens * max_deg]
  size_t d_pack;     // uint2 {u, f32 bits} [V * 4] dictionary rows padded to 4 entries (fused expansion)
  size_t a_cnt;      // int32 [sum n]
  size_t a_list;     // uint2 {lds offset, f32 bits} [src_tokens * max_deg]
  size_t a_choff;    // int32 [n_rt * (nch + 1)]
  size_t b_list;     // uint32 lds offset [tgt_tokens]
  size_t b_choff;    // int32 [n_ct * (nch + 1)]
  size_t b_mt;       // uint2 {word mask, words before} [n_ct * nch] (compacted contraction)
  size_t b_kcn;      // int32 [n_ct] compacted chunks per column tile
  size_t b_rng;      // int32 [n_ct * nch][2] first / last global chunk of each compacted chunk
  size_t a_base;     // int64 [n_rt] first A-list entry of each row tile
  size_t b_base;     // int64 [n_ct] first B-list entry of each column tile
  size_t p_voc;      // uint32 [B * ceil(V / 32)] target vocabulary of each pair (compacted contraction)
  size_t bwd;        // float [B * 4] per-pair partials + float [n_blocks * 4]
  size_t bnd;        // uint64 (value, epoch) boundary rows between strips
  size_t ctl;        // int32 [2]: DP queue head, error flag
  size_t total;
};

}  // namespace nwm
