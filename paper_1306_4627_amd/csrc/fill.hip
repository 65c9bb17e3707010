// fill.hip -- the bit-parallel fill (length, checkpoints for the traceback).
//
// Mapping: a lane keeps WPL consecutive 64-bit words of V in registers; a
// pair's words are spread over consecutive lanes.  Lane k of a pair works on
// column (t - skew_k) at step t with skew growing by one per lane, so the
// carry leaving lane k-1 for column j is produced one step before lane k
// needs it: the carry hand-over is a shift of the wave's carry-out lane mask
// (ballot) by one lane, fed back as the carry-in lane mask of the next step.
// No cross-lane add is ever waited for inside a step.
#include "kernels.hpp"
#include "bitvec.hpp"
#include "plan.hpp"

namespace lcs {

// --------------------------------------------------------------------------
// fill
// --------------------------------------------------------------------------

size_t fill_lds_bytes(int wpl, int sigma) {
    return (size_t)fill_waves(sigma, wpl) * (size_t)(sigma + 1) * (size_t)wpl * 64 * sizeof(uint64_t);
}

// Sixteen stream values (two per dword) starting at step t0.
__device__ __forceinline__ void load16(const uint16_t *ys, uint32_t t0, uint32_t (&d)[8]) {
    const uint16_t *p = ys + t0;
#pragma unroll
    for (int e = 0; e < 8; ++e) d[e] = (uint32_t)p[2 * e] | ((uint32_t)p[2 * e + 1] << 16);
}

#ifndef LCS_FILL_HOIST
#define LCS_FILL_HOIST 8
#endif

// Sixteen column steps t..t+15 of one lane.  The carry-in lane mask of a
// step is the carry-out mask of the previous step shifted up by one lane,
// with segment starts cleared; with CHAIN, lane 0 takes the hand-over bit of
// the feeding item (inbits, one bit per step) and lane 63's carry-out is
// collected into outbits for the next item.  With TB, every lane's carry-in
// bits are accumulated (newest in bit 0) and stored every 32 steps.
template <int WPL, bool TB, bool CHAIN, bool RAW>
__device__ __forceinline__ void run16(const uint32_t (&Yg)[8], uint32_t t, const char *lanecol,
                                      uint64_t notstart, uint64_t &cmask, uint32_t &acc,
                                      uint32_t *cbp, uint32_t (&vlo)[WPL], uint32_t (&vhi)[WPL],
                                      uint64_t &inbits, uint64_t &outbits) {
    constexpr int H = LCS_FILL_HOIST;   // steps whose match masks are read together
#pragma unroll
    for (int h = 0; h < 16 / H; ++h) {
        // the match masks of H steps are read up front: they depend on the
        // stream only, so their LDS latency overlaps the column steps
        uint64_t Mg[H][WPL];
#pragma unroll
        for (int e = 0; e < H; ++e) {
            const int s = h * H + e;
            const uint32_t y2 = Yg[s >> 1];
            uint32_t off = (s & 1) ? (y2 >> 16) : (y2 & 0xffffu);
            if (RAW) off <<= 9 + (WPL == 1 ? 0 : WPL == 2 ? 1 : WPL == 4 ? 2 : 3);
            const char *row = lanecol + off;
#pragma unroll
            for (int q = 0; q < WPL; ++q) Mg[e][q] = *(const uint64_t *)(row + q * 512);
        }
#pragma unroll
        for (int e = 0; e < H; ++e) {
            uint64_t cm = cmask;
            if (CHAIN) {
                cm |= inbits & 1ull;
                inbits >>= 1;
            }
            if (TB) {
                uint32_t cj;
                acc = __builtin_addc(acc, acc, (uint32_t)__builtin_amdgcn_inverse_ballot_w64(cm), &cj);
                if (h * H + e == 15 && (t & 16u)) cbp[(size_t)((t + 15) >> 5) * 64] = acc;
            }
            column_step<WPL>(vlo, vhi, Mg[e], cm);
            if (CHAIN) {
                outbits = (outbits >> 1) | (cm & 0x8000000000000000ull);
                // pin the accumulation to this step: sunk to its single use,
                // it would keep every step's carry mask alive until the chunk end
                asm volatile("" : "+s"(outbits), "+s"(inbits));
            }
            cmask = (cm << 1) & notstart;
        }
        // keep the scheduler from spreading the scalar work of many steps
        // across each other (it would hold dozens of masks live)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Y stream element: code * (WPL * 512), i.e. the byte offset of the code's
// row of match masks in the wave's LDS block ([symbol][word][lane] layout);
// with RAW the plain code, shifted here.
template <int WPL, bool TB, bool RAW>
__global__ __launch_bounds__(kFillBlock) void k_fill(FillArgs a) {
    extern __shared__ uint64_t smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int sig1 = a.sigma + 1;
    constexpr uint32_t RS = WPL * 64;            // words per symbol row
    uint64_t *pm = smem + (size_t)wv * sig1 * RS;
    // this lane's column of the wave's block; a stream value is a byte offset
    const char *lanecol = (const char *)(pm + lane);

    for (;;) {
        uint32_t ticket = 0;
        if (lane == 0) ticket = atomicAdd(a.queue, 1u);
        ticket = __builtin_amdgcn_readfirstlane(ticket);
        if (ticket >= a.item_end - a.item_begin) return;
        const uint32_t item = a.item_begin + ticket;

        const size_t li = (size_t)item * 64 + lane;
        const int32_t pair = a.ln_pair[li];
        const uint32_t word0 = a.ln_word0[li];
        const uint32_t skew = a.ln_skew[li];
        const uint64_t ysoff = a.ln_ys[li];
        const uint32_t T = a.it_T[item];
        const int32_t prev = a.it_prev[item];
        const bool feeds = a.it_feeds[item] != 0;

        // ---- match masks of this lane's rows (LDS, own column only) ----
        for (int c = 0; c < sig1; ++c)
#pragma unroll
            for (int q = 0; q < WPL; ++q) pm[c * RS + q * 64 + lane] = 0;
        uint32_t m = 0;
        if (pair >= 0) {
            m = a.pair_m[pair];
            const uint8_t *xc = a.xcodes + a.pair_xoff[pair];
            for (int q = 0; q < WPL; ++q) {
                const uint32_t row0 = (word0 + q) * 64u;
                if (row0 >= m) break;
                uint64_t *col = pm + q * 64 + lane;
                const uint32_t cnt = (m - row0) < 64u ? (m - row0) : 64u;
#pragma unroll 1
                for (uint32_t r0 = 0; r0 < cnt; r0 += 4) {
                    // the X arena is padded to 64 bytes per sequence
                    const uint32_t w4 = *(const uint32_t *)(xc + row0 + r0);
#pragma unroll
                    for (int by = 0; by < 4; ++by) {
                        const uint32_t r = r0 + by;
                        if (r < cnt) {
                            const uint32_t c = (w4 >> (8 * by)) & 0xffu;
                            atomicOr((unsigned long long *)(col + c * RS), 1ull << r);
                        }
                    }
                }
            }
        }

        // ---- column steps ----
        uint32_t vlo[WPL], vhi[WPL];
#pragma unroll
        for (int q = 0; q < WPL; ++q) { vlo[q] = ~0u; vhi[q] = ~0u; }
        const uint16_t *ys = a.ystream + ysoff - skew;
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
        bool aborted = false;
        // Stream values, two per dword, in a ring of four 16-step groups; the
        // group 32 steps ahead is requested before the current one is used,
        // so the stream's memory latency hides behind two groups of work.
        uint32_t Y0[8], Y1[8], Y2[8], Y3[8];
        load16(ys, 0, Y0);
        load16(ys, 16, Y1);
        const bool chain = prev >= 0 || feeds;
        // The longest items bound the kernel's duration: let the SIMD issue
        // their instructions first; shorter items fill the remaining slots.
        if (T >= a.prio_T) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(0);
        uint64_t pw0 = 0, pw1 = 0;   // hand-over words requested one group early

        for (uint32_t c = 0; c < nch; ++c) {
            uint64_t inbits = 0, outbits = 0;
            if (prev >= 0 && c > 0) {
                uint64_t w0 = uniform64(pw0), w1 = uniform64(pw1);
                uint32_t spins = 0;
                while ((uint32_t)(w0 >> 32) != c || (uint32_t)(w1 >> 32) != c) {
                    // bounded wait for the feeding item to finish chunk c-1
                    if (++spins > a.spin_limit) { aborted = true; break; }
                    __builtin_amdgcn_s_sleep(1);
                    w0 = uniform64(__hip_atomic_load(xf_in + 2 * (c - 1), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
                    w1 = uniform64(__hip_atomic_load(xf_in + 2 * (c - 1) + 1, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
                }
                if (aborted) break;
                inbits = (w1 << 32) | (w0 & 0xffffffffull);
            }
            if (TB && ((c * 64u) % (uint32_t)a.ckpt_every) == 0) {
                uint64_t *dst = ckp + (size_t)((c * 64u) / (uint32_t)a.ckpt_every) * RS;
#pragma unroll
                for (int q = 0; q < WPL; ++q) dst[q * 64] = ((uint64_t)vhi[q] << 32) | vlo[q];
            }
            const uint32_t t = c * 64u;
            if (chain) {
                load16(ys, t + 32, Y2);
                run16<WPL, TB, true, RAW>(Y0, t, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 48, Y3);
                run16<WPL, TB, true, RAW>(Y1, t + 16, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 64, Y0);
                run16<WPL, TB, true, RAW>(Y2, t + 32, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 80, Y1);
                if (prev >= 0) {
                    pw0 = __hip_atomic_load(xf_in + 2 * c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    pw1 = __hip_atomic_load(xf_in + 2 * c + 1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
                }
                run16<WPL, TB, true, RAW>(Y3, t + 48, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                if (feeds && lane == 0) {
                    const uint64_t tag = (uint64_t)(c + 1) << 32;
                    __hip_atomic_store(xf_out + 2 * c, tag | (outbits & 0xffffffffull),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(xf_out + 2 * c + 1, tag | (outbits >> 32), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            } else {
                load16(ys, t + 32, Y2);
                run16<WPL, TB, false, RAW>(Y0, t, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 48, Y3);
                run16<WPL, TB, false, RAW>(Y1, t + 16, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 64, Y0);
                run16<WPL, TB, false, RAW>(Y2, t + 32, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 80, Y1);
                run16<WPL, TB, false, RAW>(Y3, t + 48, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
            }
        }
        if (aborted) {
            if (lane == 0) atomicOr(a.error, 1u);
            return;
        }

        // ---- length: zero bits among the valid rows ----
        if (pair >= 0) {
            uint32_t zeros = 0;
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
            if (zeros) atomicAdd((unsigned long long *)(a.out_len + pair), (unsigned long long)zeros);
        }
    }
}

const void *fill_symbol(int wpl, bool tb, bool raw) {
    if (raw) {
        if (wpl == 1) return tb ? (const void *)&k_fill<1, true, true> : (const void *)&k_fill<1, false, true>;
        return tb ? (const void *)&k_fill<2, true, true> : (const void *)&k_fill<2, false, true>;
    }
    switch (wpl) {
        case 1: return tb ? (const void *)&k_fill<1, true, false> : (const void *)&k_fill<1, false, false>;
        case 2: return tb ? (const void *)&k_fill<2, true, false> : (const void *)&k_fill<2, false, false>;
        case 4: return tb ? (const void *)&k_fill<4, true, false> : (const void *)&k_fill<4, false, false>;
        default: return tb ? (const void *)&k_fill<8, true, false> : (const void *)&k_fill<8, false, false>;
    }
}

int fill_block(int wpl, int sigma) { return 64 * fill_waves(sigma, wpl); }

hipError_t launch_fill(int wpl, bool tb, const FillArgs &a, uint32_t grid, hipStream_t s) {
    if (!wpl_fits(a.sigma, wpl)) return hipErrorInvalidValue;
    const size_t lds = fill_lds_bytes(wpl, a.sigma);
    const dim3 block((uint32_t)fill_block(wpl, a.sigma));
    const bool raw = raw_stream(a.sigma, wpl);
#define LCS_FILL_CASE(W, R)                                                            \
    if (wpl == W && raw == R) {                                                        \
        if (tb)                                                                        \
            hipLaunchKernelGGL((k_fill<W, true, R>), dim3(grid), block, lds, s, a);    \
        else                                                                           \
            hipLaunchKernelGGL((k_fill<W, false, R>), dim3(grid), block, lds, s, a);   \
        return hipGetLastError();                                                      \
    }
    LCS_FILL_CASE(1, false)
    LCS_FILL_CASE(2, false)
    LCS_FILL_CASE(4, false)
    LCS_FILL_CASE(8, false)
    LCS_FILL_CASE(1, true)
    LCS_FILL_CASE(2, true)
#undef LCS_FILL_CASE
    return hipErrorInvalidValue;
}

}  // namespace lcs
