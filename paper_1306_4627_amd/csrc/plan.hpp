// plan.hpp -- host-side packing of LCS pairs into wave-sized work items.
//
// The fill computes, for each pair, the bit-vector form of the columns of
// the c table of section I.C: bit (i-1) of V_j is 1 exactly when
// c[i][j] == c[i-1][j] (the column does not step up at row i).  A pair with
// m rows needs W = ceil(m/64) 64-bit words per column.  A lane holds `wpl`
// consecutive words of one pair, so a pair needs s = ceil(W/wpl) lanes; the
// lanes of one pair form a "segment".
//
// Work item = one wavefront of 64 lanes.  Items are processed by persistent
// waves that take them from a queue in order.  A segment of at most 64 lanes
// lives inside one item (several segments share an item); a longer segment
// starts at lane 0 of a fresh item and continues through consecutive items
// (a "chain"), its carry bits handed from item to item through global
// memory.
//
// Diagonal skew: lane k of a segment processes column (t - skew_k) at step t,
// so the carry out of lane k-1 for column j is ready one step before lane k
// needs it.  Inside an item skew grows by 1 per lane; across an item boundary
// it grows by CHUNK, so lane 0 of the next item uses, at step t, the carry
// lane 63 of the previous item produced at step t - CHUNK: the same bit
// position of the previous chunk's hand-over word.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace lcs {

constexpr int kLanes = 64;        // lanes per work item (one wavefront)
constexpr int kChunk = 64;        // steps per chunk (carry hand-over unit)
constexpr int kCbitsPer = 32;     // steps per stored carry-in word (uint32)

struct PairShape {
    uint64_t m = 0;   // rows (|X|)
    uint64_t n = 0;   // columns (|Y|)
};

struct PlanConfig {
    int wpl = 4;            // words per lane (1, 2, 4, 8)
    bool traceback = false;
    int ckpt = 64;          // steps between stored V checkpoints (multiple of kChunk)
    int sigma = 4;          // alphabet size; code sigma is the zero-mask sentinel
    bool plain = false;     // one pair per item, no packing
    int strip_rows = 4096;  // rows per traceback strip (rounded up to whole bands)
    int link_items = 1;     // items one run of linked chains may span (1 = no sharing)
    // Traceback in rounds (0 = one pass with every item's history stored at
    // once): the fill runs once for lengths and carry hand-over words only,
    // then the items are refilled round by round, each round storing the
    // history of a set of items in one shared buffer of at most round_bytes
    // and walking the strips those items hold (see ClassPlan's rd_* tables).
    uint64_t round_bytes = 0;
    int cus = 256;          // compute units of the device (resident wave slots)
};

// A chain may start in the free lanes of the item before it when its step
// count is within this share of the largest one of the items linked to that
// item (they all run for the largest).
constexpr double kLinkSpread = 0.02;

// One class = one fill launch with a fixed words-per-lane.
struct ClassPlan {
    int wpl = 1;
    // items
    std::vector<uint32_t> it_T;       // steps, multiple of kChunk
    std::vector<int32_t> it_prev;     // item feeding lane 0 through memory, or -1
    std::vector<uint8_t> it_feeds;    // 1 if lane 63 continues into the next item
    std::vector<uint32_t> it_depth;   // items before this one in its run of linked chains
    std::vector<uint64_t> it_ck;      // checkpoint base (uint64 units)
    std::vector<uint64_t> it_cb;      // carry-bit base (uint32 units)
    std::vector<uint64_t> it_xf;      // carry hand-over base (uint64 units, 2 per chunk), for feeders
    // lanes (item-major, kLanes per item)
    std::vector<int32_t> ln_pair;     // -1 = idle
    std::vector<uint32_t> ln_word0;   // first word of the pair held by the lane
    std::vector<uint32_t> ln_skew;
    std::vector<uint64_t> ln_ys;      // Y-stream element of column 0 of the lane's segment
    uint64_t max_T = 0;
    // traceback work list for this class (sorted by cost, largest first)
    std::vector<uint32_t> tb_pair;
    std::vector<uint32_t> tb_item;    // item holding the segment's first lane
    std::vector<uint32_t> tb_lane0;   // lane of that item
    // Traceback strips.  A band is the rows one lane holds (64*wpl rows); a
    // strip is strip_bands consecutive bands of one pair, counted from row
    // 0, so a pair has S = ceil(bands / strip_bands) strips and strip S-1
    // (the top one) may be short.  Per traceback entry: its first band
    // crossing and first strip result.  Tickets: the speculative pass has
    // one per strip, the fix-up pass one per strip below the top one, the
    // seal pass one per pair with at least two strips.
    uint32_t strip_bands = 1;
    std::vector<uint32_t> tb_band0, tb_strip0;
    std::vector<uint32_t> sp_t, sp_s;   // speculative tickets: entry, strip
    std::vector<uint32_t> fx_t, fx_s;   // fix-up tickets: entry, strip
    std::vector<uint32_t> sl_t;         // seal tickets: entry
    uint64_t n_bands = 0, n_strips = 0;
    uint64_t ck_words = 0, cb_words = 0, xf_words = 0;
    uint64_t lane_steps = 0;
    // Traceback in rounds (PlanConfig::round_bytes > 0).  Every item belongs
    // to one round; a chain's items are taken top-down, so the round of an
    // item is never earlier than that of the item above it in its chain, and
    // the strips a round walks continue the path the earlier rounds wrote.
    // Per item: its round and the offset of its history in the round buffer
    // (uint64 units; V checkpoints first, then the carry-in words, so the
    // carry words of the item start at 2 * (it_rb + checkpoint words) in
    // uint32 units).  Per round r, entries [off[r], off[r+1]) of: the items
    // to refill; the speculative tickets (entry, strip; bit 31 of the strip
    // set when the strip is the top of its group below the pair's top strip
    // and starts from the column the walk left the strip above); the fix-up
    // tickets (entry, strip); the seal tickets (entry, top strip of the
    // group, bottom strip of the group).
    uint32_t n_rounds = 0;
    uint64_t round_words = 0;             // uint64 words of the round buffer
    std::vector<uint32_t> it_round;
    std::vector<uint64_t> it_rb;          // checkpoints (uint64 units)
    std::vector<uint64_t> it_rcb;         // carry-in words (uint32 units, same buffer)
    std::vector<uint32_t> rd_item_off, rd_items;
    std::vector<uint32_t> rd_sp_off, rd_sp_t, rd_sp_s;
    std::vector<uint32_t> rd_fx_off, rd_fx_t, rd_fx_s;
    std::vector<uint32_t> rd_sl_off, rd_sl_t, rd_sl_top, rd_sl_lo;
};

constexpr uint32_t kFromAbove = 0x80000000u;   // speculative ticket flag (rounds)

// One region of the Y stream: the pair's Y codes at columns 0..n-1 and the
// sentinel code elsewhere, each element scaled to a byte offset into the
// class's match-mask block (code << shift).  A region with pair == kNoPair
// is all sentinel; idle lanes of the class read it.
constexpr uint32_t kNoPair = 0xffffffffu;
struct Segment {
    uint32_t pair;
    uint64_t begin;     // first element of the region
    uint32_t pre;       // sentinel elements before column 0
    uint64_t len;       // region length in elements
    uint8_t shift;      // log2(words_per_lane * 512)
};

struct Plan {
    PlanConfig cfg;
    std::vector<ClassPlan> classes;
    std::vector<Segment> segs;
    uint64_t ys_elems = 0;        // total Y-stream elements (uint16)
    uint64_t cells = 0;
    uint64_t items = 0;
    uint64_t lanes = 0;
    uint64_t lane_steps = 0;
    uint64_t max_T = 0;
    std::vector<uint32_t> pair_class;   // class of each pair (UINT32_MAX if empty)
};

// Largest number of rows a pair may have for a given words-per-lane
// (a segment may span at most kMaxChain items).
constexpr int kMaxChain = 4096;
inline uint64_t max_rows(int wpl) { return (uint64_t)kMaxChain * kLanes * wpl * 64; }

// Largest words-per-lane the kernels accept for an alphabet size, and
// whether a given one fits (stream element width and LDS size); whether the
// stream holds plain codes (alphabets too large for pre-shifted ones); and
// the fill's waves per work-group.
int max_wpl(int sigma);
bool wpl_fits(int sigma, int wpl);
bool raw_stream(int sigma, int wpl);
int fill_waves(int sigma, int wpl);

// Build a plan.  Returns an empty string on success, else a reason.
std::string build_plan(const std::vector<PairShape> &pairs, const PlanConfig &cfg, Plan &out);

// Structural checks of a plan (used by tests through the C ABI).
std::string check_plan(const std::vector<PairShape> &pairs, const Plan &p);

}  // namespace lcs
