// fill.hip -- the bit-parallel fill (length, checkpoints for the traceback).
//
// Mapping: a lane keeps WPL consecutive 64-bit words of V in registers; a
// pair's words are spread over consecutive lanes.  Lane k of a pair works on
// column (t - skew_k) at step t with skew growing by one per lane, so the
// carry leaving lane k-1 for column j is produced one step before lane k
// needs it: the carry hand-over is a shift of the wave's carry-out lane mask
// (ballot) by one lane, fed back as the carry-in lane mask of the next step.
// No cross-lane add is ever waited for inside a step.
#include <algorithm>

#include "kernels.hpp"
#include "bitvec.hpp"
#include "plan.hpp"

namespace lcs {

// --------------------------------------------------------------------------
// fill
// --------------------------------------------------------------------------

size_t fill_lds_bytes(int wpl, int sigma, int mode) {
    const size_t waves = (size_t)fill_waves(sigma, wpl);
    // match masks: [symbol + sentinel][word][lane] per wave; the threshold
    // pass adds 128 32-bit words per wave (segment sums and answers)
    return waves * (size_t)(sigma + 1) * (size_t)wpl * 64 * sizeof(uint64_t) +
           (mode == kFillThreshold ? waves * 128 * sizeof(uint32_t) : 0);
}

// Sixteen stream values (two per dword) starting at step t0.
__device__ __forceinline__ void load16(const uint16_t *ys, uint32_t t0, uint32_t (&d)[8]) {
    const uint16_t *p = ys + t0;
#pragma unroll
    for (int e = 0; e < 8; ++e) d[e] = (uint32_t)p[2 * e] | ((uint32_t)p[2 * e + 1] << 16);
}

// Match masks of eight steps (steps s0..s0+7 of a group of sixteen stream
// values): they depend on the stream only, so they are read from LDS ahead
// of the column steps that use them.
template <int WPL, bool RAW>
__device__ __forceinline__ void read_masks8(const uint32_t (&Yg)[8], int s0, const char *lanecol,
                                            uint64_t (&M)[8][WPL]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int s = s0 + e;
        const uint32_t y2 = Yg[s >> 1];
        uint32_t off = (s & 1) ? (y2 >> 16) : (y2 & 0xffffu);
        if (RAW) off <<= 9 + (WPL == 1 ? 0 : WPL == 2 ? 1 : WPL == 4 ? 2 : 3);
        const char *row = lanecol + off;
#pragma unroll
        for (int q = 0; q < WPL; ++q) M[e][q] = *(const uint64_t *)(row + q * 512);
    }
}

// Eight column steps t+8h..t+8h+7 of one lane, with their match masks.  The
// carry-in lane mask of a step is the carry-out mask of the previous step
// shifted up by one lane, with segment starts cleared.  With CHAIN, lane 0
// takes the hand-over bit of the feeding item and lane 63's carry-out is
// collected for the next item: one scalar add-with-carry chain shifts the
// mask (2 * mask, the carry into the low word being the next step's hand-over
// bit, selected by s_bitcmp1 from `innext`, bit s = the bit of step s+1) and
// shifts lane 63's carry (bit 63 of the mask, the chain's carry out) into
// `ow` (most recent step in bit 0).  (Collected by plain code instead, the
// lengths-only fill at two words per lane spilled some 100 SGPRs into VGPR
// lanes and had its match-mask reads sunk next to their steps.)  With TB,
// every lane's carry-in bits are accumulated (newest in bit 0: acc = 2 * acc
// + carry-in, one v_addc_co_u32 with the mask as carry-in) and stored every
// 32 steps.
template <int WPL, bool TB, bool CHAIN>
__device__ __forceinline__ void steps8(const uint64_t (&Mg)[8][WPL], int h, uint32_t t,
                                       uint64_t notstart, uint64_t &cmask, uint32_t &acc,
                                       uint32_t *cbp, uint32_t (&vlo)[WPL], uint32_t (&vhi)[WPL],
                                       uint32_t innext, uint32_t &ow) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        uint64_t cm = cmask;
        if (TB) {
            asm("v_addc_co_u32 %[a], vcc, %[a], %[a], %[m]" : [a] "+v"(acc) : [m] "s"(cm) : "vcc");
            if (h * 8 + e == 15 && (t & 16u)) cbp[(size_t)((t + 15) >> 5) * 64] = acc;
        }
        column_step<WPL>(vlo, vhi, Mg[e], cm);
        if (CHAIN) {
            const uint32_t clo = (uint32_t)cm, chi = (uint32_t)(cm >> 32);
            uint32_t lo, hi;
            asm("s_bitcmp1_b32 %[in], %[bit]\n\t"
                "s_addc_u32 %[lo], %[clo], %[clo]\n\t"
                "s_addc_u32 %[hi], %[chi], %[chi]\n\t"
                "s_addc_u32 %[ow], %[ow], %[ow]"
                : [lo] "=&s"(lo), [hi] "=&s"(hi), [ow] "+s"(ow)
                : [in] "s"(innext), [bit] "i"(h * 8 + e), [clo] "s"(clo), [chi] "s"(chi)
                : "scc");
            cmask = (((uint64_t)hi << 32) | lo) & notstart;
        } else {
            cmask = (cm << 1) & notstart;
        }
    }
}

// Sixteen column steps t..t+15 of one lane, the match masks of each eight
// steps read just before them.
template <int WPL, bool TB, bool CHAIN, bool RAW>
__device__ __forceinline__ void run16(const uint32_t (&Yg)[8], uint32_t t, const char *lanecol,
                                      uint64_t notstart, uint64_t &cmask, uint32_t &acc,
                                      uint32_t *cbp, uint32_t (&vlo)[WPL], uint32_t (&vhi)[WPL],
                                      uint32_t innext, uint32_t &ow) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint64_t Mg[8][WPL];
        read_masks8<WPL, RAW>(Yg, 8 * h, lanecol, Mg);
        // (without this barrier the scheduler may sink each read to its
        // step, and every step then waits out a whole LDS latency)
        __builtin_amdgcn_sched_barrier(0);
        steps8<WPL, TB, CHAIN>(Mg, h, t, notstart, cmask, acc, cbp, vlo, vhi, innext, ow);
        // keep the scheduler from spreading the scalar work of many steps
        // across each other (it would hold dozens of masks live)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One chunk: 64 column steps t..t+63, four groups of sixteen stream values
// in a ring (Y0, Y1 hold the chunk's first two groups on entry; the group 32
// steps ahead is requested before each group runs, so on return Y0, Y1 hold
// the next chunk's first two).  `inbits`: with CHAIN, the hand-over bits of
// the chunk (bit s = step s); ow_lo, ow_hi receive lane 63's carries of the
// chunk's two halves.  (Reading each eight steps' match masks while the
// eight before them run, with two sets of mask registers, measured no faster
// on short protein pairs and 2-6% slower on the related DNA batch, whose
// lengths-only fill it took from four waves per SIMD to three.)
template <int WPL, bool TB, bool CHAIN, bool RAW>
__device__ __forceinline__ void run64(uint32_t (&Y0)[8], uint32_t (&Y1)[8], uint32_t (&Y2)[8],
                                      uint32_t (&Y3)[8], const uint16_t *ys, uint32_t t,
                                      const char *lanecol, uint64_t notstart, uint64_t &cmask,
                                      uint32_t &acc, uint32_t *cbp, uint32_t (&vlo)[WPL],
                                      uint32_t (&vhi)[WPL], uint64_t inbits, uint32_t &ow_lo,
                                      uint32_t &ow_hi) {
    const uint32_t in0 = (uint32_t)(inbits >> 1), in1 = (uint32_t)(inbits >> 17);
    const uint32_t in2 = (uint32_t)(inbits >> 33), in3 = (uint32_t)(inbits >> 49);
    load16(ys, t + 32, Y2);
    run16<WPL, TB, CHAIN, RAW>(Y0, t, lanecol, notstart, cmask, acc, cbp, vlo, vhi, in0, ow_lo);
    load16(ys, t + 48, Y3);
    run16<WPL, TB, CHAIN, RAW>(Y1, t + 16, lanecol, notstart, cmask, acc, cbp, vlo, vhi, in1, ow_lo);
    load16(ys, t + 64, Y0);
    run16<WPL, TB, CHAIN, RAW>(Y2, t + 32, lanecol, notstart, cmask, acc, cbp, vlo, vhi, in2, ow_hi);
    load16(ys, t + 80, Y1);
    run16<WPL, TB, CHAIN, RAW>(Y3, t + 48, lanecol, notstart, cmask, acc, cbp, vlo, vhi, in3, ow_hi);
}

// Zero bits among this lane's valid rows of V: the lane's share of
// c[m][j] for the column it holds (rows above m are padding).
template <int WPL>
__device__ __forceinline__ uint32_t lane_zeros(const uint32_t (&vlo)[WPL], const uint32_t (&vhi)[WPL],
                                               int32_t pair, uint32_t word0, uint32_t m) {
    uint32_t zeros = 0;
    if (pair >= 0) {
#pragma unroll
        for (int q = 0; q < WPL; ++q) {
            const uint32_t row0 = (word0 + q) * 64u;
            if (row0 < m) {
                const uint32_t cnt = (m - row0) < 64u ? (m - row0) : 64u;
                const uint64_t mask = cnt == 64u ? ~0ull : ((1ull << cnt) - 1);
                const uint64_t v = ((uint64_t)vhi[q] << 32) | vlo[q];
                zeros += cnt - (uint32_t)__builtin_popcountll(v & mask);
            }
        }
    }
    return zeros;
}

// Answer word of a pair (relaxed, device scope: other waves set it).  Idle
// lanes read pair 0's word and report 0; no branch, so the load can sit
// between column steps without splitting the wave's control flow.
__device__ __forceinline__ uint32_t load_state(uint32_t *dec, int32_t pair) {
    const uint32_t d = __hip_atomic_load(dec + (pair >= 0 ? pair : 0), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return pair >= 0 ? d : 0u;
}

__device__ __forceinline__ uint32_t clamp_col(int64_t j, uint32_t n) {
    return j <= 0 ? 0u : (j >= (int64_t)n ? n : (uint32_t)j);
}

// Y stream element: code * (WPL * 512), i.e. the byte offset of the code's
// row of match masks in the wave's LDS block ([symbol][word][lane] layout);
// with RAW the plain code, shifted here.
//
// MODE kFillThreshold (section II's yes/no question: does the child keep at
// least a given share of the parent?): at the start of every kThrEvery-th
// chunk each lane counts the zero bits of its rows, the counts are summed per
// pair segment of the wave, and a chained item adds the running sum handed up
// by the item below (taken at the start of that item's previous chunk) and
// hands the new sum up with its carries.  An item d places into its run of
// linked chains checks at the chunks c with c = d (mod kThrEvery), so its
// feeder checked at chunk c - 1.
// The one-chunk delay per item offsets the item's 64 extra steps of skew, so
// the sum H seen by a pair's top lane covers every row block at columns
// falling by one per lane from Jb (bottom lane) to J (top lane).  Column steps raise c by at most one, hence
// H - (Jb - J) <= c[m][J] <= H, and since c[m][n] >= c[m][J] and
// c[m][n] <= c[m][J] + (n - J), the pair reaches its target T once
// H - (Jb - J) >= T and cannot once H + (n - J) < T.  The top lane then
// records the answer; a wave whose pairs are all answered stops, and so do
// the items of a chain once its pair is.
constexpr uint32_t kThrEvery = 4;   // chunks between threshold checks of an item

// Queue place of a wave's next item (lane 0 only).  The queue holds the items
// longest first; left alone, the waves starting together take the first
// places in no particular order, and a SIMD may get several of the longest
// items at once: its waves then share its issue until the end of the pass
// while other SIMDs run out of work.  With bands, a wave's first item is the
// next place of band r, r its rank among this launch's waves on its SIMD, so
// each SIMD starts with one item of each band.  Later items (and a first item
// whose band is used up) come from places the bands left untaken, bands in
// order, then from the places after the bands.  Every place is taken once;
// places of one band go out in order, and a band's leftovers before any later
// place, so an item's feeder (the place before it) has been taken first or is
// among the few leftovers the next free wave takes.
__device__ __forceinline__ uint32_t next_place(const FillArgs &a, bool first) {
    const uint32_t B = a.band_size;
    if (!B) return atomicAdd(a.queue, 1u);
    if (first) {
        const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID
        const uint32_t xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // XCC_ID
        const uint32_t key = ((xcc & 15u) << 10) | (((hw >> 13) & 7u) << 7) |
                             (((hw >> 12) & 1u) << 6) | (((hw >> 8) & 15u) << 2) | ((hw >> 4) & 3u);
        const uint32_t r = atomicAdd(a.simd_rank + key, 1u);
        if (r < a.nbands) {
            const uint32_t q = atomicAdd(a.band_next + r, 1u);
            if (q < B) return r * B + q;
        }
    }
    for (uint32_t k = 0; k < a.nbands; ++k) {
        if (__hip_atomic_load(a.band_next + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < B) {
            const uint32_t q = atomicAdd(a.band_next + k, 1u);
            if (q < B) return k * B + q;
        }
    }
    return a.nbands * B + atomicAdd(a.queue, 1u);
}

template <int WPL, int MODE, bool RAW>
__device__ __forceinline__ void fill_body(const FillArgs &a) {
    constexpr bool TB = MODE == kFillTraceback;
    constexpr bool THR = MODE == kFillThreshold;
    extern __shared__ uint64_t smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int sig1 = a.sigma + 1;
    constexpr uint32_t RS = WPL * 64;            // words per symbol row
    uint64_t *pm = smem + (size_t)wv * sig1 * RS;
    // this lane's column of the wave's block; a stream value is a byte offset
    const char *lanecol = (const char *)(pm + lane);
    // threshold pass: 64 segment sums and 64 segment answers per wave
    uint32_t *tslot = nullptr;
    if (THR) tslot = (uint32_t *)(smem + (size_t)(blockDim.x >> 6) * sig1 * RS) + wv * 128;
    // the clock during the fill: shader cycles over 100 MHz ticks of the
    // first wave's lifetime
    const bool clk_lane = a.clk && blockIdx.x == 0 && threadIdx.x == 0;
    if (clk_lane) {
        a.clk[0] = __builtin_amdgcn_s_memtime();
        a.clk[1] = __builtin_amdgcn_s_memrealtime();
    }

    bool first = true;
    for (;;) {
        uint32_t ticket = 0;
        if (lane == 0) ticket = next_place(a, first);
        first = false;
        ticket = __builtin_amdgcn_readfirstlane(ticket);
        if (ticket >= a.item_end - a.item_begin) {
            if (clk_lane) {
                a.clk[2] = __builtin_amdgcn_s_memtime();
                a.clk[3] = __builtin_amdgcn_s_memrealtime();
            }
            return;
        }
        const uint32_t item = a.item_list ? a.item_list[a.item_begin + ticket] : a.item_begin + ticket;
        const uint64_t taken = a.trace ? __builtin_amdgcn_s_memrealtime() : 0;

        const size_t li = (size_t)item * 64 + lane;
        const int32_t pair = a.ln_pair[li];
        const uint32_t word0 = a.ln_word0[li];
        const uint32_t skew = a.ln_skew[li];
        const uint64_t ysoff = a.ln_ys[li];
        const uint32_t T = a.it_T[item];
        const int32_t prev = a.it_prev[item];
        const bool feeds = a.it_feeds[item] != 0;

        // the first two groups of stream values are requested now: their
        // latency overlaps the match-mask build
        const uint16_t *ys = a.ystream + ysoff - skew;
        uint32_t Y0[8], Y1[8], Y2[8], Y3[8];
        load16(ys, 0, Y0);
        load16(ys, 16, Y1);

        // ---- match masks of this lane's rows (LDS, own column only) ----
        for (int c = 0; c < sig1; ++c)
#pragma unroll
            for (int q = 0; q < WPL; ++q) pm[c * RS + q * 64 + lane] = 0;
        uint32_t m = 0;
        if (pair >= 0) {
            m = a.pair_m[pair];
            const uint8_t *xc = a.xcodes + a.pair_xoff[pair];
#pragma unroll
            for (int q = 0; q < WPL; ++q) {
                const uint32_t row0 = (word0 + q) * 64u;
                if (row0 >= m) continue;
                // the word's 64 codes with four 16-byte loads issued together
                // (each sequence starts 64-byte aligned in the X arena and is
                // padded to a multiple of 64 bytes)
                const uint4 *src = (const uint4 *)(xc + row0);
                const uint4 d0 = src[0], d1 = src[1], d2 = src[2], d3 = src[3];
                // rows past m set no bit: the bit of row r is masked with the
                // word's valid rows, so every row is one 32-bit LDS OR into
                // its half of the code's mask word, without a branch
                const uint32_t cnt = (m - row0) < 64u ? (m - row0) : 64u;
                const uint32_t ok_lo = cnt >= 32u ? ~0u : ((1u << cnt) - 1u);
                const uint32_t ok_hi = cnt >= 64u ? ~0u : cnt <= 32u ? 0u : ((1u << (cnt - 32u)) - 1u);
                char *col = (char *)(pm + q * 64 + lane);
                const uint32_t w[16] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w,
                                        d2.x, d2.y, d2.z, d2.w, d3.x, d3.y, d3.z, d3.w};
#pragma unroll
                for (int r = 0; r < 64; ++r) {
                    const uint32_t c = (w[r >> 2] >> (8 * (r & 3))) & 0xffu;
                    uint32_t *dst = (uint32_t *)(col + c * (RS * 8u)) + (r >> 5);
                    atomicOr(dst, (r < 32 ? ok_lo : ok_hi) & (1u << (r & 31)));
                }
            }
        }

        // ---- column steps ----
        if (a.trace && lane == 0) {
            a.trace[(size_t)item * kTraceWords] = taken;
            a.trace[(size_t)item * kTraceWords + 1] = __builtin_amdgcn_s_memrealtime();
        }
        uint32_t vlo[WPL], vhi[WPL];
#pragma unroll
        for (int q = 0; q < WPL; ++q) { vlo[q] = ~0u; vhi[q] = ~0u; }
        const uint64_t startmask = __builtin_amdgcn_ballot_w64(pair < 0 || word0 == 0);
        const uint64_t notstart = ~startmask;
        uint64_t cmask = 0;
        uint32_t acc = 0;
        const uint32_t nch = T / 64;
        uint64_t *ckp = nullptr;
        uint32_t *cbp = nullptr;
        if (TB) {
            ckp = a.ckpt + a.it_ck[item] + lane;
            cbp = a.cbits + a.it_cb[item] + lane;
        }
        // Carry hand-over between chained items: chunk c of a feeder is two
        // 64-bit words, each a 32-bit tag (c + 1) above 32 carry bits, written
        // with relaxed agent-scope atomic stores; the consumer accepts a word
        // once its tag matches.  The words carry their own validity, so no
        // release/acquire fence (an L2 write-back on this chip) is needed;
        // the buffer is zeroed before every pass.
        uint64_t *xf_out = feeds ? a.xfer + a.it_xf[item] : nullptr;
        uint64_t *xf_in = prev >= 0 ? a.xfer + a.it_xf[prev] : nullptr;
        // threshold pass: the running sums travel the same way, one tagged
        // word per chunk
        uint64_t *xs_out = (THR && feeds) ? a.xsum + a.it_xf[item] / 2 : nullptr;
        const uint64_t *xs_in = (THR && prev >= 0) ? a.xsum + a.it_xf[prev] / 2 : nullptr;
        // threshold pass: this lane's segment (first lane, top lane) and the
        // state of its pair; `live_in` drops once the chained pair entering
        // at lane 0 is answered (nothing more needs to come from below)
        int seg0 = 0;
        bool seg_top = false;
        uint32_t nq = 0, tq = 0, pdec = 0, pdec_nx = 0;
        bool live_in = prev >= 0;
        // check phase: the item's place in its run of linked chains (every
        // feeder sits one place below the item it feeds)
        uint32_t phase = 0;
        if (THR) {
            phase = a.it_depth[item] % kThrEvery;
            const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
            seg0 = 63 - __builtin_clzll((startmask | 1ull) & upto);
            const int32_t pair_up = __shfl(pair, lane == 63 ? 63 : lane + 1);
            seg_top = pair >= 0 && (lane == 63 || pair_up != pair);
            if (pair >= 0) {
                nq = a.pair_n[pair];
                tq = a.thr_t[pair];
            }
            pdec = load_state(a.thr_dec, pair);
        }
        bool aborted = false, stopped = false;
        // Stream values, two per dword, in a ring of four 16-step groups (the
        // first two were requested above); the group 32 steps ahead is
        // requested before the current one is used, so the stream's memory
        // latency hides behind two groups of work.
        const bool chain = prev >= 0 || feeds;
        uint64_t pw0 = 0, pw1 = 0, pw2 = 0;   // hand-over words requested one chunk early
        uint64_t waited = 0;                   // schedule record: ticks spent waiting

        for (uint32_t c = 0; c < nch; ++c) {
            // Wave priority by the column steps left (longest remaining
            // first), re-set every 16th chunk: the SIMD issues first for the
            // waves with the most work left, so its waves tend to finish
            // together and it keeps several of them to hide latency until its
            // last item ends (a fixed priority for the longest items left the
            // items taken later, at default priority, to end the pass).
            // Levels at half, a quarter and an eighth of the longest item.
            // (Re-set every fourth chunk, short items kept trading places:
            // 5% slower on batches of short pairs.)
            if ((c & 15u) == 0) {
                const uint32_t rem = T - c * 64u, h = a.prio_half;
                if (rem >= h) __builtin_amdgcn_s_setprio(3);
                else if (2 * rem >= h) __builtin_amdgcn_s_setprio(2);
                else if (4 * rem >= h) __builtin_amdgcn_s_setprio(1);
                else __builtin_amdgcn_s_setprio(0);
            }
            uint64_t inbits = 0;
            uint32_t hin = 0;
            if (live_in && c > 0) {
                uint64_t w0 = uniform64(pw0), w1 = uniform64(pw1), w2 = THR ? uniform64(pw2) : 0;
                uint32_t spins = 0;
                // (the running sum is handed up only for this item's check chunks)
                const bool want_sum = THR && (c + kThrEvery - phase) % kThrEvery == 0;
                const bool late = (uint32_t)(w0 >> 32) != c || (uint32_t)(w1 >> 32) != c ||
                                  (want_sum && (uint32_t)(w2 >> 32) != c);
                const uint64_t wait0 = (a.trace && late) ? __builtin_amdgcn_s_memrealtime() : 0;
                while ((uint32_t)(w0 >> 32) != c || (uint32_t)(w1 >> 32) != c ||
                       (want_sum && (uint32_t)(w2 >> 32) != c)) {
                    // bounded wait for the feeding item to finish chunk c-1
                    if (++spins > a.spin_limit) { aborted = true; break; }
                    if (THR) {
                        // the pair may have been answered, and the feeder gone
                        const uint32_t d = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                            a.thr_dec + __builtin_amdgcn_readfirstlane(pair), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT));
                        if (d) { stopped = true; break; }
                    }
                    __builtin_amdgcn_s_sleep(1);
                    w0 = uniform64(__hip_atomic_load(xf_in + 2 * (c - 1), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
                    w1 = uniform64(__hip_atomic_load(xf_in + 2 * (c - 1) + 1, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
                    if (want_sum)
                        w2 = uniform64(__hip_atomic_load(xs_in + (c - 1), __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT));
                }
                if (wait0) waited += __builtin_amdgcn_s_memrealtime() - wait0;
                if (aborted || stopped) break;
                inbits = (w1 << 32) | (w0 & 0xffffffffull);
                hin = (uint32_t)w2;
                cmask |= inbits & 1ull;   // lane 0's carry-in of the chunk's first step
            }
            const uint32_t t = c * 64u;
            uint32_t hout = 0;
            // this item's check chunks; its sum word is handed up at each of
            // them (at chunk 0 it is 0: no column is done yet)
            const bool sum_chunk = THR && (c + kThrEvery - phase) % kThrEvery == 0;
            const bool check = sum_chunk && c > 0;
            if (THR) {
                if (!pdec) pdec = pdec_nx;
                if (check) {
                    // segment sums of the zero counts (LDS, in wave order)
                    const uint32_t z = lane_zeros<WPL>(vlo, vhi, pair, word0, m);
                    tslot[lane] = 0;
                    tslot[64 + lane] = 0;
                    wave_lds_sync();
                    atomicAdd(tslot + seg0, z);
                    wave_lds_sync();
                    uint32_t h = tslot[seg0];
                    if (seg0 == 0 && prev >= 0) h += hin;
                    hout = __builtin_amdgcn_readlane(h, 63);
                    if (seg_top && pdec == 0 && !(lane == 63 && feeds)) {
                        // this lane tops its pair: columns J (own) and Jb
                        // (bottom lane, `below` item boundaries and as many
                        // chunks earlier; lane g of a pair has a skew of g
                        // plus kChunk - 1 per boundary below it)
                        const uint32_t J = clamp_col((int64_t)t - (int64_t)skew, nq);
                        const uint32_t below = (skew - word0 / WPL) / (uint32_t)(kChunk - 1);
                        const uint32_t Jb = clamp_col(64 * ((int64_t)c - (int64_t)below), nq);
                        uint32_t d = 0;
                        if ((uint64_t)h >= (uint64_t)tq + (Jb - J)) d = 1;
                        else if ((uint64_t)h + (nq - J) < (uint64_t)tq) d = 2;
                        if (d) {
                            __hip_atomic_store(a.thr_dec + pair, d, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            tslot[64 + seg0] = d;
                        }
                    }
                    wave_lds_sync();
                    const uint32_t dl = tslot[64 + seg0];
                    if (dl && pair >= 0) pdec = dl;
                }
                // every pair of the wave answered: stop
                if (__builtin_amdgcn_ballot_w64(pair >= 0 && pdec == 0) == 0) {
                    stopped = true;
                    break;
                }
                // the chained pair at lane 0 answered: stop waiting for it
                if (live_in && __builtin_amdgcn_readlane(pdec, 0) != 0) live_in = false;
            }
            // The hand-over words of this chunk (used at the start of the next
            // one) and the pair states are requested now, a whole chunk ahead:
            // a device-scope load takes about as long as a chunk of a wave
            // that has its SIMD to itself, so a later request would stall the
            // next chunk's start.  Words not yet written are polled again.
            // With the traceback history, these two reads and the checkpoint
            // store below are issued on every path -- an item with no feeder
            // reads, and a chunk with no checkpoint writes, the junk words --
            // so that the compiler counts them in its memory-counter waits for
            // the stream reads issued before them; under a branch they made it
            // wait for everything outstanding, the hand-over reads just
            // requested included (the 262144-row pair's traceback fill: 5%
            // slower).  The lengths-only fill keeps the branch: issued on
            // every path, the reads moved its full wait to the chunk start,
            // where it catches the stream read issued 16 steps earlier (3%
            // slower on a SIMD of its own, the same with four waves).
            if (TB || live_in) {
                const uint64_t *src = live_in ? xf_in + 2 * c : a.junk;
                pw0 = __hip_atomic_load(const_cast<uint64_t *>(src), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
                pw1 = __hip_atomic_load(const_cast<uint64_t *>(src) + 1, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
            }
            if (THR && live_in && (c + 1 + kThrEvery - phase) % kThrEvery == 0)
                pw2 = __hip_atomic_load(xs_in + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (THR) pdec_nx = load_state(a.thr_dec, pair);
            if (TB) {
                const bool ck = ((c * 64u) % (uint32_t)a.ckpt_every) == 0;
                uint64_t *dst = ck ? ckp + (size_t)((c * 64u) / (uint32_t)a.ckpt_every) * RS : a.junk + lane;
#pragma unroll
                for (int q = 0; q < WPL; ++q) dst[q * 64] = ((uint64_t)vhi[q] << 32) | vlo[q];
            }
            if (chain) {
                // hand-over bits of the next step: bit s of each group's word
                // is the bit of step (group start + s + 1) of the chunk
                uint32_t ow_lo = 0, ow_hi = 0;
                run64<WPL, TB, true, RAW>(Y0, Y1, Y2, Y3, ys, t, lanecol, notstart, cmask, acc,
                                                cbp, vlo, vhi, inbits, ow_lo, ow_hi);
                // lane 63's carries of the chunk, step e in bit e
                const uint64_t outbits =
                    ((uint64_t)__builtin_bitreverse32(ow_hi) << 32) | __builtin_bitreverse32(ow_lo);
                if (feeds && lane == 0) {
                    const uint64_t tag = (uint64_t)(c + 1) << 32;
                    __hip_atomic_store(xf_out + 2 * c, tag | (outbits & 0xffffffffull),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(xf_out + 2 * c + 1, tag | (outbits >> 32), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    if (sum_chunk)
                        __hip_atomic_store(xs_out + c, tag | hout, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            } else {
                uint32_t dummy_lo = 0, dummy_hi = 0;
                run64<WPL, TB, false, RAW>(Y0, Y1, Y2, Y3, ys, t, lanecol, notstart, cmask, acc,
                                                 cbp, vlo, vhi, 0ull, dummy_lo, dummy_hi);
            }
        }
        if (a.trace && lane == 0) {
            uint64_t *r = a.trace + (size_t)item * kTraceWords;
            r[2] = __builtin_amdgcn_s_memrealtime();
            r[3] = waited;
            // HW_ID and XCC_ID, all 32 bits of each
            r[4] = ((uint64_t)__builtin_amdgcn_s_getreg((31 << 11) | 4) << 32) |
                   __builtin_amdgcn_s_getreg((31 << 11) | 20);
        }
        if (aborted) {
            if (lane == 0) atomicOr(a.error, 1u);
            return;
        }
        // an answered pair's length is not needed (and not complete)
        if (THR && stopped) continue;

        // ---- length: zero bits among the valid rows ----
        if (!a.out_len) continue;
        // a half of a split pair keeps its last column for the combine (the
        // split is for lengths-only batches; compiled into the other modes,
        // this store alone made the traceback fill 11% slower)
        const bool half = MODE == kFillLength && a.out_v && pair >= (int32_t)a.v_pair0;
        if (half) {
            uint64_t *dst = a.out_v + a.pair_vbase[pair - (int32_t)a.v_pair0];
#pragma unroll
            for (int q = 0; q < WPL; ++q)
                if ((word0 + q) * 64u < m) dst[word0 + q] = ((uint64_t)vhi[q] << 32) | vlo[q];
        }
        const uint32_t zeros = half ? 0u : lane_zeros<WPL>(vlo, vhi, pair, word0, m);
        if (zeros) atomicAdd((unsigned long long *)(a.out_len + pair), (unsigned long long)zeros);
    }
}

// Kernel entry points.  Left to itself the compiler gives the threshold mode
// about 150 VGPRs at two words per lane (three waves per SIMD); held to 128
// at one or two words per lane it keeps four waves like the lengths-only
// fill, and the values that then spill belong to the per-item set-up and the
// threshold checks, not to the column steps (5% faster on the 4096-pair
// related batch).  The traceback mode (132 VGPRs) measured 5% slower when
// held to 128, and wider lanes would spill inside the steps: both keep the
// unconstrained entry.
template <int WPL, int MODE, bool RAW>
__global__ __launch_bounds__(kFillBlock) void k_fill(FillArgs a) {
    fill_body<WPL, MODE, RAW>(a);
}

template <int WPL, int MODE, bool RAW>
__global__ __launch_bounds__(kFillBlock) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_fill4(FillArgs a) {
    fill_body<WPL, MODE, RAW>(a);
}

template <int WPL, int MODE, bool RAW>
static const void *fill_entry() {
    if constexpr (WPL <= 2 && MODE == kFillThreshold) return (const void *)&k_fill4<WPL, MODE, RAW>;
    else return (const void *)&k_fill<WPL, MODE, RAW>;
}

const void *fill_symbol(int wpl, int mode, bool raw, int sigma) {
    (void)sigma;
#define LCS_FILL_SYM(W, R)                                                              \
    if (wpl == W && raw == R) {                                                         \
        if (mode == kFillTraceback) return fill_entry<W, kFillTraceback, R>();          \
        if (mode == kFillThreshold) return fill_entry<W, kFillThreshold, R>();          \
        return fill_entry<W, kFillLength, R>();                                         \
    }
    LCS_FILL_SYM(1, false)
    LCS_FILL_SYM(2, false)
    LCS_FILL_SYM(4, false)
    LCS_FILL_SYM(8, false)
    LCS_FILL_SYM(1, true)
    LCS_FILL_SYM(2, true)
#undef LCS_FILL_SYM
    return nullptr;
}

int fill_block(int wpl, int sigma) { return 64 * fill_waves(sigma, wpl); }

hipError_t launch_fill(int wpl, int mode, const FillArgs &a, uint32_t grid, hipStream_t s) {
    if (!wpl_fits(a.sigma, wpl)) return hipErrorInvalidValue;
    if (mode == kFillThreshold && (!a.pair_n || !a.thr_t || !a.thr_dec || !a.xsum))
        return hipErrorInvalidValue;
    const void *fn = fill_symbol(wpl, mode, raw_stream(a.sigma, wpl), a.sigma);
    if (!fn) return hipErrorInvalidValue;
    FillArgs arg = a;
    void *args[] = {&arg};
    return hipLaunchKernel(fn, dim3(grid), dim3((uint32_t)fill_block(wpl, a.sigma)), args,
                           fill_lds_bytes(wpl, a.sigma, mode), s);
}

}  // namespace lcs
