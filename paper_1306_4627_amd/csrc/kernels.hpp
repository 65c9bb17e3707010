// kernels.hpp -- argument blocks and launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lcs {

// One region of the Y stream, as the stream builder reads it (32 bytes,
// one pair of 16-byte loads).
struct SegInfo {
    uint64_t begin;   // first element of the region
    uint64_t yoff;    // offset of its pair's Y in the Y arena
    uint32_t len;     // region length in elements
    uint32_t pre;     // sentinel elements before column 0
    uint32_t n;       // columns of its pair (0 for an all-sentinel region)
    uint32_t shift;   // log2 of the stream scale (words_per_lane * 512), or 0;
                      // plus kSegReversed: column c holds Y[n - 1 - c]
};

constexpr uint32_t kSegReversed = 0x100;

// A pair whose length comes from two fills of half its columns each: X
// against Y[0, h), and X reversed against Y[h, n) reversed.  The reversed X
// codes are written by the prep launch; the fill stores the last column of
// both halves; k_halves combines them.
struct HalfInfo {
    uint64_t xsrc;    // the pair's X in the X arena (bytes)
    uint64_t xdst;    // its reversed codes in the X-code arena
    uint64_t vf;      // last column of the first half in the column buffer (words)
    uint64_t vb;      // last column of the reversed second half
    uint32_t pair;    // the pair whose length is written
    uint32_t m;       // rows
};

// Symbol remap and Y-stream construction (all device pointers).
struct PrepArgs {
    const uint8_t *lut;        // 256 entries: byte -> code (validated on the host)
    const uint8_t *xbytes;     // X arena (raw bytes)
    uint8_t *xcodes;           // X arena (codes), same offsets
    uint64_t xarena;           // bytes in the X arena
    const uint8_t *ybytes;     // Y arena (raw bytes)
    const SegInfo *seg;        // stream regions
    uint32_t nseg;
    const uint32_t *blk_seg;   // region of each 64-element block of the stream
    uint64_t nblk;             // 64-element blocks in the stream (regions are
                               // whole blocks, laid out back to back)
    uint16_t *ystream;         // element = code << seg_shift
    uint32_t sentinel;         // code whose match mask is zero (= alphabet size)
    uint64_t *out_len;         // zeroed here (per pair)
    uint32_t npairs;
    uint32_t *zero_words;      // counters/flags zeroed here
    uint64_t nzero;
    uint64_t *zero64;          // traceback bitmaps zeroed here
    uint64_t nzero64;
    // threshold pass (null otherwise): the state word of each pair is set
    // here from its target: 1 for a target of 0, 2 for one above min(m, n)
    // (both settled before any column), else 0
    const uint32_t *pair_m;
    const uint32_t *pair_n;
    const uint32_t *thr_t;
    uint32_t *thr_dec;
    // split pairs (null when none): the reversed X codes of each
    const HalfInfo *halves;
    uint32_t nhalves;
};

// Fill: one class (fixed words per lane), persistent waves.
struct FillArgs {
    const uint8_t *xcodes;
    const uint64_t *pair_xoff;
    const uint32_t *pair_m;
    const uint16_t *ystream;   // per class: code * (words_per_lane * 512)
    const uint32_t *it_T;
    const int32_t *it_prev;
    const uint8_t *it_feeds;
    const uint32_t *it_depth;  // items before this one in its run of linked chains
    const uint64_t *it_ck;
    const uint64_t *it_cb;
    const uint64_t *it_xf;
    const int32_t *ln_pair;
    const uint32_t *ln_word0;
    const uint32_t *ln_skew;
    const uint64_t *ln_ys;
    uint64_t *out_len;         // null: lengths not added (traceback rounds' refills)
    // halves of split pairs: pairs from v_pair0 on store their last column
    // at out_v + pair_vbase[pair - v_pair0] instead of adding a length
    uint64_t *out_v;
    const uint64_t *pair_vbase;
    uint32_t v_pair0;
    uint64_t *ckpt;
    uint32_t *cbits;
    uint64_t *xfer;            // hand-over words, two per chunk per feeder (zeroed)
    uint32_t *queue;           // work counter (zeroed before the launch)
    // First-item bands (optional, band_size 0 = off): the first nbands *
    // band_size queue places form nbands bands; a wave's first item is the
    // next place of the band of its rank among the launch's waves on its
    // SIMD (simd_rank: kSimdKeys counters, band_next: kMaxBands counters,
    // all zeroed before the launch), so that every SIMD starts with one item
    // of each band instead of several of the longest ones
    uint32_t *simd_rank;
    uint32_t *band_next;
    uint32_t band_size;
    uint32_t nbands;
    uint32_t *error;           // set to 1 when a bounded wait runs out
    // kJunkWords words of any content: the chunk-start reads of an item with
    // no feeder and the checkpoint stores of chunks that keep none go here
    uint64_t *junk;
    uint32_t item_begin;
    uint32_t item_end;
    // optional: the items to run are item_list[item_begin .. item_end)
    // instead of the range itself (traceback rounds refill a set of items)
    const uint32_t *item_list;
    uint32_t prio_half;        // half the longest item's steps: scale of the wave priorities
    uint32_t spin_limit;       // polls before a wait gives up
    int32_t sigma;             // code sigma is the zero-mask sentinel
    int32_t ckpt_every;        // steps between checkpoints (traceback only)
    // threshold pass only
    const uint32_t *pair_n;    // columns of each pair
    const uint32_t *thr_t;     // target length of each pair
    uint32_t *thr_dec;         // 0 open, 1 reaches its target, 2 cannot
    uint64_t *xsum;            // running zero counts handed up a chain: one
                               // tagged word per chunk per feeder (zeroed)
    // optional: the shader-clock and 100 MHz counters read by the first wave
    // of work-group 0 when it starts and when it finds the queue empty
    uint64_t *clk;
    // optional schedule record of every item (kTraceWords words, zeroed
    // before the pass): 100 MHz counter when the item is taken from the
    // queue, at its first column step and after its last one; counter ticks
    // spent waiting for the feeding item's carries; HW_ID (high half) and
    // XCC_ID (low half) of the wave that ran it
    uint64_t *trace;
};

constexpr int kTraceWords = 6;
constexpr uint32_t kJunkWords = 8 * 64;   // eight words per lane

// First-item bands: SIMD keys from HW_ID and XCC_ID (XCC 4 bits, shader
// engine 3, shader array 1, CU 4, SIMD 2) and the most bands of a launch.
constexpr uint32_t kSimdKeys = 1u << 14;
constexpr uint32_t kMaxBands = 8;

// What a fill launch computes: lengths only, lengths plus the checkpoints the
// traceback reads, or the threshold pass (lengths of the pairs it does not
// settle early).
enum FillMode { kFillLength = 0, kFillTraceback = 1, kFillThreshold = 2 };

// Traceback walk: one wave per ticket, persistent.  The walk records the
// rows where it takes a diagonal step in a per-pair bitmap over X (bit r of
// word w stands for row 64*w + r + 1); k_emit turns the bitmap into bytes.
struct TbArgs {
    const uint8_t *xcodes;
    const uint64_t *pair_xoff;
    const uint32_t *pair_m;
    const uint32_t *pair_n;
    const uint64_t *pair_diag;  // first bitmap word of each pair
    uint64_t *diag;             // bitmaps (zeroed before the launch)
    const uint16_t *ystream;    // per class: code * (words_per_lane * 512)
    const uint32_t *it_T;
    const uint64_t *it_ck;
    const uint64_t *it_cb;
    const uint32_t *ln_skew;
    const uint64_t *ln_ys;
    const uint64_t *ckpt;
    const uint32_t *cbits;
    const uint32_t *tb_pair;    // per traceback entry: pair
    const uint32_t *tb_item;    //   item holding its first lane
    const uint32_t *tb_lane0;   //   lane of that item
    const uint32_t *tb_band0;   //   first entry of its band crossings
    const uint32_t *tb_strip0;  //   first entry of its strip results
    const uint32_t *tk_t;       // per ticket: traceback entry
    const uint32_t *tk_s;       // per ticket: strip (speculative and fix-up passes;
                                // speculative with kFromAbove: the strip starts at
                                // the column the walk left the strip above); seal
                                // pass: top strip of the group, or null for the
                                // pair's top strip
    const uint32_t *tk_lo;      // seal pass: bottom strip of the group, or null for 0
    uint32_t nticket;
    uint32_t *queue;
    uint32_t *cross;            // per band: column where the speculative walk leaves it
    uint32_t *strip_res;        // per strip: {entry column of the fix-up, exit column}
    uint32_t strip_bands;       // bands per strip
    int32_t mode;               // kTbSpec, kTbFix or kTbSeal
    int32_t sigma;
    int32_t ckpt_every;
    int32_t nb;                 // tiles per band recomputed together (one per lane)
    int32_t nbands;             // bands per recompute round
    int32_t ysh;                // stream value >> ysh = symbol code
};

// Traceback passes over strips (runs of bands of one pair): speculative
// walks from estimated entry columns, fix-up walks from the speculative exit
// of the strip above until they rejoin the speculative path, and one
// sequential seal per pair.
enum : int32_t { kTbSpec = 0, kTbFix = 1, kTbSeal = 2 };

// Emit: bitmap of diagonal rows -> LCS bytes (X symbols in row order), one
// item per 64 bitmap words of a pair.
struct EmitArgs {
    const uint8_t *xbytes;
    const uint64_t *pair_xoff;
    const uint32_t *pair_m;
    const uint32_t *pair_n;
    const uint64_t *pair_diag;
    const uint64_t *diag;
    const uint64_t *pair_out;
    const uint64_t *out_len;
    uint8_t *out;
    const uint32_t *em_pair;    // per item: pair
    const uint32_t *em_w0;      // per item: first of its (up to) 64 bitmap words
    uint32_t nitems;
    uint32_t *error;            // set to 2 when a bitmap disagrees with the length
};

// Combine of split pairs: one work-group per pair.
struct HalvesArgs {
    const HalfInfo *halves;
    uint32_t nhalves;
    const uint64_t *v;         // last columns of the halves
    uint64_t *out_len;
};

constexpr int kFillBlock = 256;   // at most four independent waves per work-group
constexpr int kTbBlock = 256;

size_t fill_lds_bytes(int wpl, int sigma, int mode);
// LDS of a traceback work-group of `waves` waves (1..4, one wave per ticket)
size_t tb_lds_bytes(int wpl, int sigma, int ckpt_every, int nb, int bands, int waves = 4);

const void *fill_symbol(int wpl, int mode, bool raw, int sigma);
int fill_block(int wpl, int sigma);   // threads per fill work-group
const void *tb_symbol(int wpl, int ckpt_every);

hipError_t launch_prep(const PrepArgs &a, uint64_t xbytes_n, hipStream_t s);
hipError_t launch_fill(int wpl, int mode, const FillArgs &a, uint32_t grid, hipStream_t s);
hipError_t launch_tb(int wpl, const TbArgs &a, uint32_t grid, int waves, hipStream_t s);
hipError_t launch_emit(const EmitArgs &a, hipStream_t s);
hipError_t launch_halves(const HalvesArgs &a, hipStream_t s);

}  // namespace lcs
