// lcs_kernels.hip -- gfx950 kernels of the LCS library.
//
// Bit-vector form of the dynamic program of section I.C.  For column j let
// V_j be the m-bit vector whose bit (i-1) is 1 exactly when
// c[i][j] == c[i-1][j].  Column 0 is all zero in c, so V_0 is all ones; with
// PM_a the match mask of symbol a (bit (i-1) set when x_i == a), one column
// step is the add-and-mask recurrence of Allison & Dix (1986) in the
// four-operation form of Crochemore, Iliopoulos, Pinzon & Reid (2001):
//
//     U = V & PM[y_j]        V' = (V + U) | (V & ~PM[y_j])
//
// where "+" is an m-bit addition whose carries run from row 1 upward.  Then
// c[i][j] = i - popcount(V_j & (2^i - 1)), so the LCS length c[m][n] is the
// number of zero bits among the m valid bits of V_n.
//
// Mapping: a lane keeps WPL consecutive 64-bit words of V in registers; a
// pair's words are spread over consecutive lanes.  Lane k of a pair works on
// column (t - skew_k) at step t with skew growing by one per lane, so the
// carry leaving lane k-1 for column j is produced one step before lane k
// needs it: the carry hand-over is a shift of the wave's carry-out lane mask
// (ballot) by one lane, fed back as the carry-in lane mask of the next step.
// No cross-lane add is ever waited for inside a step.
//
// Traceback (section I.D with ties going up): at (i, j) a match moves
// diagonally and emits x_i; otherwise c[i-1][j] >= c[i][j-1] holds exactly
// when c[i-1][j] == c[i][j], i.e. when bit (i-1) of V_j is 1, and the walk
// moves up; else it moves left.  Inside one column the walk therefore jumps
// to the highest row r <= i with (PM[y_j] | ~V_j) set at r.  The fill stores
// V every `ckpt_every` steps and every lane's carry-in bits, so any
// (lane, step range) tile of the V history can be recomputed on its own;
// the traceback recomputes only the tiles the path crosses.
#include "kernels.hpp"

namespace lcs {

// --------------------------------------------------------------------------
// prep: symbol remap (bytes -> codes), Y streams, zeroing
// --------------------------------------------------------------------------

__global__ void k_remap_x(const uint8_t *__restrict__ lut, const uint8_t *__restrict__ src,
                          uint8_t *__restrict__ dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 4;
    for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
        if (i + 4 <= n) {
            uint32_t w = *(const uint32_t *)(src + i);
            uint32_t r = (uint32_t)lut[w & 0xff] | ((uint32_t)lut[(w >> 8) & 0xff] << 8) |
                         ((uint32_t)lut[(w >> 16) & 0xff] << 16) | ((uint32_t)lut[w >> 24] << 24);
            *(uint32_t *)(dst + i) = r;
        } else {
            for (uint64_t k = i; k < n; ++k) dst[k] = lut[src[k]];
        }
    }
}

// One work-group per stream region (grid-stride over regions): codes of Y at
// columns 0..n-1, the sentinel code everywhere else in the region, each
// shifted into a byte offset of its row of match masks.
__global__ __launch_bounds__(256) void k_streams(PrepArgs a) {
    // the byte -> code table in LDS; each thread writes eight stream values
    // (16 bytes, aligned: regions start at multiples of 64 elements and are
    // padded to them) per pass, and gridDim.y blocks share a region
    __shared__ uint8_t lut[256];
    lut[threadIdx.x] = a.lut[threadIdx.x];
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.y * blockDim.x * 8;
    for (uint32_t s = blockIdx.x; s < a.nseg; s += gridDim.x) {
        const uint64_t begin = a.seg_begin[s];
        const uint64_t len = a.seg_len[s];
        const uint64_t pre = a.seg_pre[s];
        const uint64_t n = a.seg_n[s];
        const uint32_t sh = a.seg_shift[s];
        const uint8_t *y = a.ybytes + a.seg_yoff[s];
        const uint32_t sent = (uint32_t)a.sentinel << sh;
        for (uint64_t k0 = ((uint64_t)blockIdx.y * blockDim.x + threadIdx.x) * 8; k0 < len; k0 += stride) {
            uint32_t c[8];
            if (k0 >= pre && k0 + 8 <= pre + n) {
                // eight bytes of Y from two aligned 8-byte reads (the Y arena
                // is padded by 64 bytes)
                const uintptr_t ad = (uintptr_t)(y + (k0 - pre));
                const uint64_t *al = (const uint64_t *)(ad & ~(uintptr_t)7);
                const uint32_t s8 = (uint32_t)(ad & 7) * 8;
                const uint64_t lo = al[0], hi = al[1];
                const uint64_t v = s8 ? (lo >> s8) | (hi << (64 - s8)) : lo;
#pragma unroll
                for (int e = 0; e < 8; ++e) c[e] = (uint32_t)(v >> (8 * e)) & 0xffu;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint64_t k = k0 + e;
                    c[e] = (k >= pre && k - pre < n) ? (uint32_t)y[k - pre] : 0x100u;
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) c[e] = c[e] == 0x100u ? sent : ((uint32_t)lut[c[e]] << sh);
            uint4 v;
            v.x = c[0] | (c[1] << 16);
            v.y = c[2] | (c[3] << 16);
            v.z = c[4] | (c[5] << 16);
            v.w = c[6] | (c[7] << 16);
            *(uint4 *)(a.ystream + begin + k0) = v;
        }
    }
}

__global__ void k_zero(PrepArgs a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = tid; k < a.npairs; k += stride) a.out_len[k] = 0;
    for (uint64_t k = tid; k < a.nzero; k += stride) a.zero_words[k] = 0;
    for (uint64_t k = tid; k < a.nzero64; k += stride) a.zero64[k] = 0;
}

hipError_t launch_prep(const PrepArgs &a, uint64_t xbytes_n, hipStream_t s) {
    if (xbytes_n) {
        uint64_t blocks = (xbytes_n / 4 + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_remap_x, dim3((uint32_t)blocks), dim3(256), 0, s, a.lut, a.xbytes,
                           a.xcodes, xbytes_n);
    }
    hipLaunchKernelGGL(k_zero, dim3(512), dim3(256), 0, s, a);
    if (a.nseg) {
        uint32_t blocks = a.nseg < 65536 ? a.nseg : 65536;
        hipLaunchKernelGGL(k_streams, dim3(blocks, 8), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// fill
// --------------------------------------------------------------------------

size_t fill_lds_bytes(int wpl, int sigma) {
    return (size_t)(kFillBlock / 64) * (size_t)(sigma + 1) * (size_t)wpl * 64 * sizeof(uint64_t);
}

// One column step for WPL words of one lane: U = V & M, S = V + U + carry
// (64*WPL-bit add, carry in and out as a wave lane mask in an SGPR pair),
// V' = S | (V & ~M).  Six VALU instructions per 64 cells.
//
// The carry mask is written by a VALU instruction (v_addc_co_u32) and read
// by the next v_addc_co_u32; gfx950 needs two wait states between the two,
// which the order below provides with independent instructions: inside a
// word the low-half bitop3 and the high-half AND sit between the two adds;
// across words the high-half bitop3 of the previous word and the low-half
// AND of the next one do.  The carry mask coming in is always written by
// scalar instructions and the one going out is only read by scalar
// instructions, which need no wait states.
template <int WPL>
__device__ __forceinline__ void column_step(uint32_t (&vlo)[WPL], uint32_t (&vhi)[WPL],
                                            const uint64_t (&M)[WPL], uint64_t &carry) {
#pragma unroll
    for (int q = 0; q < WPL; ++q) {
        const uint32_t mlo = (uint32_t)M[q], mhi = (uint32_t)(M[q] >> 32);
        uint32_t t0, t1;
        asm("v_and_b32 %[ulo], %[vlo], %[mlo]\n\t"
            "v_addc_co_u32 %[ulo], %[c], %[vlo], %[ulo], %[c]\n\t"
            "v_bitop3_b32 %[vlo], %[ulo], %[vlo], %[mlo] bitop3:0xf4\n\t"
            "v_and_b32 %[uhi], %[vhi], %[mhi]\n\t"
            "v_addc_co_u32 %[uhi], %[c], %[vhi], %[uhi], %[c]\n\t"
            "v_bitop3_b32 %[vhi], %[uhi], %[vhi], %[mhi] bitop3:0xf4"
            : [vlo] "+v"(vlo[q]), [vhi] "+v"(vhi[q]), [c] "+s"(carry), [ulo] "=&v"(t0),
              [uhi] "=&v"(t1)
            : [mlo] "v"(mlo), [mhi] "v"(mhi));
    }
}

// Make a value the compiler cannot prove wave-uniform live in SGPRs again (a
// no-op when it already does).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
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
template <int WPL, bool TB, bool CHAIN>
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
            const uint32_t off = (s & 1) ? (y2 >> 16) : (y2 & 0xffffu);
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
// row of match masks in the wave's LDS block ([symbol][word][lane] layout).
template <int WPL, bool TB>
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
                run16<WPL, TB, true>(Y0, t, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 48, Y3);
                run16<WPL, TB, true>(Y1, t + 16, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 64, Y0);
                run16<WPL, TB, true>(Y2, t + 32, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 80, Y1);
                if (prev >= 0) {
                    pw0 = __hip_atomic_load(xf_in + 2 * c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    pw1 = __hip_atomic_load(xf_in + 2 * c + 1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
                }
                run16<WPL, TB, true>(Y3, t + 48, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                if (feeds && lane == 0) {
                    const uint64_t tag = (uint64_t)(c + 1) << 32;
                    __hip_atomic_store(xf_out + 2 * c, tag | (outbits & 0xffffffffull),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(xf_out + 2 * c + 1, tag | (outbits >> 32), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            } else {
                load16(ys, t + 32, Y2);
                run16<WPL, TB, false>(Y0, t, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 48, Y3);
                run16<WPL, TB, false>(Y1, t + 16, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 64, Y0);
                run16<WPL, TB, false>(Y2, t + 32, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
                load16(ys, t + 80, Y1);
                run16<WPL, TB, false>(Y3, t + 48, lanecol, notstart, cmask, acc, cbp, vlo, vhi, inbits, outbits);
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

const void *fill_symbol(int wpl, bool tb) {
    switch (wpl) {
        case 1: return tb ? (const void *)&k_fill<1, true> : (const void *)&k_fill<1, false>;
        case 2: return tb ? (const void *)&k_fill<2, true> : (const void *)&k_fill<2, false>;
        case 4: return tb ? (const void *)&k_fill<4, true> : (const void *)&k_fill<4, false>;
        default: return tb ? (const void *)&k_fill<8, true> : (const void *)&k_fill<8, false>;
    }
}

hipError_t launch_fill(int wpl, bool tb, const FillArgs &a, uint32_t grid, hipStream_t s) {
    const size_t lds = fill_lds_bytes(wpl, a.sigma);
#define LCS_FILL_CASE(W)                                                                  \
    case W:                                                                               \
        if (tb)                                                                           \
            hipLaunchKernelGGL((k_fill<W, true>), dim3(grid), dim3(kFillBlock), lds, s, a); \
        else                                                                              \
            hipLaunchKernelGGL((k_fill<W, false>), dim3(grid), dim3(kFillBlock), lds, s, a); \
        break;
    switch (wpl) {
        LCS_FILL_CASE(1)
        LCS_FILL_CASE(2)
        LCS_FILL_CASE(4)
        LCS_FILL_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef LCS_FILL_CASE
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// traceback
// --------------------------------------------------------------------------

// Per-wave LDS of the walk, in 64-bit words.  A recompute round covers up
// to `bands` consecutive bands with `nb` tiles each (a slot per tile): the
// bands' match masks, the V words of every slot (each slot padded by two
// words so that the slots start in different LDS banks), the slots' stream
// values and carry-in words, and per band the first and last resident tile.
__host__ __device__ static inline size_t tb_slot_words(int wpl, int K) { return (size_t)K * wpl + 2; }

// Every region starts on a 16-byte boundary (an even word count before it).
__host__ __device__ static inline size_t tb_even(size_t w) { return (w + 1) & ~(size_t)1; }

__host__ __device__ static inline size_t tb_wave_words(int wpl, int sigma, int K, int nb, int bands) {
    const size_t slots = (size_t)nb * bands;
    return tb_even((size_t)bands * (sigma + 1) * wpl) + slots * tb_slot_words(wpl, K) +
           tb_even(slots * K / 4) + tb_even(slots * K / 64) + tb_even((size_t)bands);
}

size_t tb_lds_bytes(int wpl, int sigma, int K, int nb, int bands) {
    return (size_t)(kTbBlock / 64) * tb_wave_words(wpl, sigma, K, nb, bands) * sizeof(uint64_t);
}

// Lane `idx` (wave-uniform) of a 64-bit per-lane value, as a scalar.
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int32_t idx) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, idx);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), idx);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// V of one band over the 2^LOGK steps of one tile, from the checkpoint V0
// before its first step: the fill's column recurrence with the stored
// carry-in bits (most significant bit first, one 32-bit word per 32 steps),
// V after every step stored to dst.  The carry-in bit of a step becomes the
// carry lane mask by adding the carry word to itself (its top bit is the
// carry out); two wait states follow that VALU write before the first add
// reads the mask.
template <int WPL, int LOGK>
__device__ __forceinline__ void recompute_tile(uint64_t *dst, const uint64_t *pmd, const uint16_t *yst,
                                               const uint32_t *cbs, const uint64_t (&V0)[WPL]) {
    constexpr uint32_t K = 1u << LOGK;
    constexpr uint32_t kShift = 9 + (WPL == 1 ? 0 : WPL == 2 ? 1 : WPL == 4 ? 2 : 3);
    uint32_t vlo[WPL], vhi[WPL];
#pragma unroll
    for (int q = 0; q < WPL; ++q) {
        vlo[q] = (uint32_t)V0[q];
        vhi[q] = (uint32_t)(V0[q] >> 32);
    }
    for (uint32_t o0 = 0; o0 < K; o0 += 32) {
        uint32_t cw = cbs[o0 >> 5];
#pragma unroll
        for (uint32_t o1 = 0; o1 < 32; o1 += 8) {
            // eight stream values in one 16-byte read, then all eight steps'
            // match masks before any store of this group
            const uint4 y8 = *(const uint4 *)(yst + o0 + o1);
            const uint32_t yw[4] = {y8.x, y8.y, y8.z, y8.w};
            uint64_t Mg[8][WPL];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t code = ((k & 1) ? (yw[k >> 1] >> 16) : (yw[k >> 1] & 0xffffu)) >> kShift;
#pragma unroll
                for (int q = 0; q < WPL; ++q) Mg[k][q] = pmd[code * WPL + q];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                uint64_t carry;
                asm("v_add_co_u32 %[cw], %[c], %[cw], %[cw]\n\t"
                    "s_nop 1"
                    : [cw] "+v"(cw), [c] "=s"(carry));
                column_step<WPL>(vlo, vhi, Mg[k], carry);
                uint64_t *d = dst + (size_t)(o0 + o1 + k) * WPL;
#pragma unroll
                for (int q = 0; q < WPL; ++q) d[q] = ((uint64_t)vhi[q] << 32) | vlo[q];
            }
        }
    }
}

// The walk of section I.D: inside column j the walk climbs to the highest
// row r <= i whose bit is set in PM[y_j] | ~V_j; a match there is a diagonal
// step (emit x_r, go to (r-1, j-1)), otherwise the column steps left at r.
// The walk is a function of its position alone, so two walks that reach one
// position coincide from there on.  V_j for the rows of a band (the rows one
// lane of the fill held) is recomputed from the fill's checkpoints in tiles
// of 2^LOGK steps, one lane per tile, each from its own checkpoint and the
// band's stored carry-in bits.  A round recomputes nb tiles for each of up
// to nbands bands below the walk's position: the tiles ending at the walk's
// column for the band it is in, and for the next bands the tiles around the
// column the straight line from (0, 0) to (m, n) predicts for them.  A band
// whose tiles miss the walk starts a new round.
//
// A pair's rows are cut into strips of strip_bands bands, counted from row
// 0.  Three passes, one launch each:
//  - speculative: every strip is walked at once, the top strip from (m, n),
//    the others from their top row and the column the straight line crosses
//    it at; each records the column at which it leaves every band;
//  - fix-up: every strip below the top one is walked again from the column
//    the speculative walk of the strip above left it at, band by band, until
//    it leaves a band at the same column as the speculative walk of this
//    strip (from there on the two walks coincide) -- unless it starts there;
//  - seal: per pair, from the top, the exit of each strip is the entry of the
//    next; a strip whose fix-up started elsewhere is walked again whole.
// Every walk rewrites the bitmap words of the bands it crosses.
template <int WPL, int LOGK>
__global__ __launch_bounds__(kTbBlock) void k_traceback(TbArgs a) {
    extern __shared__ uint64_t smem[];
    constexpr uint32_t K = 1u << LOGK;
    constexpr uint32_t BAND = 64u * WPL;
    constexpr uint32_t kShift = 9 + (WPL == 1 ? 0 : WPL == 2 ? 1 : WPL == 4 ? 2 : 3);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int32_t sig1 = a.sigma + 1;
    const int32_t NB = a.nb;
    const int32_t NBD = a.nbands;
    const uint32_t SW = (uint32_t)tb_slot_words(WPL, (int)K);
    uint64_t *pm = smem + (size_t)wv * tb_wave_words(WPL, a.sigma, (int)K, NB, NBD);  // [band][sig1][WPL]
    const size_t NS = (size_t)NB * NBD;                                               // slots
    uint64_t *tiles = pm + tb_even((size_t)NBD * sig1 * WPL);                          // [slot][K][WPL] + pad
    uint16_t *ystage = (uint16_t *)(tiles + NS * SW);                                  // [slot][K]
    uint32_t *cbstage = (uint32_t *)((uint64_t *)ystage + tb_even(NS * K / 4));        // [slot][K/32]
    int2 *bmeta = (int2 *)((uint64_t *)cbstage + tb_even(NS * K / 64));              // [band] {lo, hi}
    const int32_t G = (int32_t)a.strip_bands;
    const int32_t R = G * (int32_t)BAND;                      // rows per strip
    const int32_t margin = NB * (int32_t)K / 4;

    for (;;) {
        uint32_t ticket = 0;
        if (lane == 0) ticket = atomicAdd(a.queue, 1u);
        ticket = __builtin_amdgcn_readfirstlane(ticket);
        if (ticket >= a.nticket) return;
        const uint32_t te = a.tk_t[ticket];
        const uint32_t p = a.tb_pair[te];
        const uint32_t item0 = a.tb_item[te];
        const uint32_t lane0 = a.tb_lane0[te];
        const uint32_t m = a.pair_m[p];
        const uint32_t n = a.pair_n[p];
        const uint8_t *xc = a.xcodes + a.pair_xoff[p];
        uint64_t *dg = a.diag + a.pair_diag[p];
        uint32_t *cross = a.cross + a.tb_band0[te];
        uint32_t *sres = a.strip_res + 2 * (size_t)a.tb_strip0[te];
        const int32_t S = (int32_t)((m + (uint32_t)R - 1) / (uint32_t)R);
        int32_t s = a.mode == kTbSeal ? S - 2 : (int32_t)a.tk_s[ticket];
        // seal: exit column of the strip above the current one
        int32_t e = a.mode == kTbSeal ? (int32_t)cross[(S - 1) * G] : 0;

        for (;;) {
            const int32_t top = (s + 1) * R;       // first row above strip s
            // column at which the speculative walk enters strip s
            const uint32_t guess_raw = (uint32_t)(((uint64_t)(uint32_t)top * n) / m);
            const int32_t guess = guess_raw < 1u ? 1 : (int32_t)guess_raw;
            int32_t i = top, j = 0;
            bool walk = true;
            const bool rec = a.mode == kTbSpec;    // record band crossings
            const bool cmp = a.mode == kTbFix;     // stop where the speculative walk is met
            if (a.mode == kTbSpec) {
                if (s == S - 1) {
                    i = (int32_t)m;
                    j = (int32_t)n;
                } else {
                    j = guess;
                }
            } else if (a.mode == kTbFix) {
                e = (int32_t)cross[(s + 1) * G];
                j = e;
                walk = e != guess;
            } else {
                j = e;
                walk = (int32_t)sres[2 * s] != e;
            }
            const int32_t i_stop = s * R;
            bool merged = false;
            if (walk) {
                int32_t band = -1, rtop = -1, nbr = 0, dsl = 0, klo = 0, khi = -1;
                uint32_t skew = 0;
                int32_t dwi = -1;          // bitmap word being filled
                uint64_t dword = 0;
                // per-band data of up to 64 bands md_lo.. (lane g: band
                // md_lo + g): skew, stream offset of step 0, checkpoint and
                // carry-bit offsets, carry words stored
                const int32_t band_lo = i_stop / (int32_t)BAND;
                int32_t md_lo = 0x7fffffff;
                uint32_t v_skew = 0, v_tw = 0;
                uint64_t v_yso = 0, v_cko = 0, v_cbo = 0;
                while (i > i_stop && j > 0) {
                    const int32_t ell = (i - 1) / (int32_t)BAND;
                    if (ell != band) {
                        band = ell;
                        if (ell < md_lo || (ell - NBD + 1 < md_lo && md_lo > band_lo)) {
                            md_lo = ell - 63 > band_lo ? ell - 63 : band_lo;
                            const int32_t bg = md_lo + lane;
                            if (bg <= ell) {
                                const uint32_t g = lane0 + (uint32_t)bg;
                                const uint32_t it = item0 + g / 64;
                                const uint32_t ln = g % 64;
                                const size_t li = (size_t)it * 64 + ln;
                                v_skew = a.ln_skew[li];
                                v_yso = a.ln_ys[li] - v_skew;
                                v_cko = a.it_ck[it] + ln;
                                v_cbo = a.it_cb[it] + ln;
                                v_tw = a.it_T[it] / 32;
                            }
                        }
                        skew = (uint32_t)__builtin_amdgcn_readlane((int32_t)v_skew, ell - md_lo);
                        const int32_t d = rtop - ell;
                        if (d >= 0 && d < nbr) {
                            dsl = d;
                            const int2 mt = bmeta[d];
                            klo = __builtin_amdgcn_readfirstlane(mt.x);
                            khi = __builtin_amdgcn_readfirstlane(mt.y);
                        } else {
                            klo = 0;
                            khi = -1;
                        }
                    }
                    const int32_t t = (j - 1) + (int32_t)skew;
                    const int32_t kt = t >> LOGK;
                    if (kt > khi || kt < klo) {
                        // a new round over bands ell, ell-1, ..., ell-nbr+1
                        rtop = ell;
                        nbr = ell - band_lo + 1;
                        nbr = nbr < NBD ? nbr : NBD;
                        const int32_t ns = nbr * NB;
                        // each slot lane u < ns: band u/NB's last tile, from
                        // the walk's column for the band it is in and from the
                        // straight line for the bands below, then tile - u%NB
                        int32_t kts = -1, khs = 0, kls = 0;
                        uint64_t yoff = 0, cko = 0, cbo = 0;
                        uint32_t tws = 0;
                        {
                            // the band data of each slot's band, read from the
                            // lane holding it (all lanes take part in the reads)
                            const int32_t d = lane / NB;
                            int32_t src = ell - d - md_lo;
                            src = src < 0 ? 0 : (src > 63 ? 63 : src);
                            const uint32_t skd = (uint32_t)__shfl((int32_t)v_skew, src, 64);
                            const uint64_t yso = ((uint64_t)(uint32_t)__shfl((int32_t)(v_yso >> 32), src, 64) << 32) |
                                                 (uint32_t)__shfl((int32_t)v_yso, src, 64);
                            const uint64_t ckd = ((uint64_t)(uint32_t)__shfl((int32_t)(v_cko >> 32), src, 64) << 32) |
                                                 (uint32_t)__shfl((int32_t)v_cko, src, 64);
                            const uint64_t cbd = ((uint64_t)(uint32_t)__shfl((int32_t)(v_cbo >> 32), src, 64) << 32) |
                                                 (uint32_t)__shfl((int32_t)v_cbo, src, 64);
                            const uint32_t twd = (uint32_t)__shfl((int32_t)v_tw, src, 64);
                            if (lane < ns) {
                                khs = kt;
                                if (d > 0) {
                                    // rows from here to band ell-d's top row, at
                                    // the straight line's slope
                                    const int64_t rows = (int64_t)i - (int64_t)(ell - d + 1) * (int64_t)BAND;
                                    int64_t c = (int64_t)j - rows * (int64_t)n / (int64_t)m + margin;
                                    c = c > j ? j : c;
                                    c = c < 1 ? 1 : c;
                                    khs = (int32_t)((c - 1 + (int64_t)skd) >> LOGK);
                                }
                                kls = khs - NB + 1 < 0 ? 0 : khs - NB + 1;
                                kts = khs - lane % NB;
                                if (kts < kls) kts = -1;
                                yoff = yso + ((uint64_t)(kts < 0 ? 0 : kts) << LOGK);
                                cko = ckd;
                                cbo = cbd;
                                tws = twd;
                            }
                        }
                        // every global read of the round first: the rows of
                        // the bands (match masks), the slots' checkpoints,
                        // stream values and carry words
                        uint64_t V0[WPL];
#pragma unroll
                        for (int q = 0; q < WPL; ++q)
                            V0[q] = kts >= 0 ? a.ckpt[cko + ((size_t)kts * WPL + q) * 64] : 0ull;
                        constexpr int kRowReads = 8;      // rows read per lane in one batch
                        constexpr uint32_t kYPerSlot = K / 2;   // stream values per slot, in pairs
                        const int32_t nrows = nbr * (int32_t)BAND;
                        const int32_t nyv = ns * (int32_t)kYPerSlot;
                        const int32_t ncb = ns * (int32_t)(K / 32);
                        uint32_t xr[kRowReads], yv[8], cv[2];
#pragma unroll
                        for (int k = 0; k < kRowReads; ++k) {
                            const int32_t r = lane + 64 * k;
                            const uint32_t row = (uint32_t)(ell - r / (int32_t)BAND) * BAND + (uint32_t)(r % (int32_t)BAND);
                            xr[k] = (r < nrows && row < m) ? (uint32_t)xc[row] : 0xffffffffu;
                        }
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const int32_t x = lane + 64 * k;
                            const int32_t u = x / (int32_t)kYPerSlot;
                            const uint64_t yo = ((uint64_t)(uint32_t)__shfl((int32_t)(yoff >> 32), u & 63, 64) << 32) |
                                                (uint32_t)__shfl((int32_t)yoff, u & 63, 64);
                            const bool ok = x < nyv && __shfl(kts, u & 63, 64) >= 0;
                            const uint16_t *ysrc = a.ystream + yo + 2 * (uint32_t)(x % (int32_t)kYPerSlot);
                            yv[k] = ok ? ((uint32_t)ysrc[0] | ((uint32_t)ysrc[1] << 16)) : 0u;
                        }
#pragma unroll
                        for (int k = 0; k < 2; ++k) {
                            const int32_t x = lane + 64 * k;
                            const int32_t u = x / (int32_t)(K / 32);
                            const uint64_t cb0 = ((uint64_t)(uint32_t)__shfl((int32_t)(cbo >> 32), u & 63, 64) << 32) |
                                                 (uint32_t)__shfl((int32_t)cbo, u & 63, 64);
                            const int32_t ku = __shfl(kts, u & 63, 64);
                            const uint32_t tw = (uint32_t)__shfl((int32_t)tws, u & 63, 64);
                            const uint32_t w = ((uint32_t)ku << (LOGK - 5)) + (uint32_t)(x % (int32_t)(K / 32));
                            cv[k] = (x < ncb && ku >= 0 && w < tw) ? a.cbits[cb0 + (size_t)w * 64] : 0u;
                        }
                        // match masks of the round's bands
                        for (int32_t u = lane; u < nbr * sig1 * WPL; u += 64) pm[u] = 0;
                        if (lane < ns && lane % NB == 0) bmeta[lane / NB] = make_int2(kls, khs);
                        wave_lds_sync();
#pragma unroll
                        for (int k = 0; k < kRowReads; ++k) {
                            const int32_t r = lane + 64 * k;
                            if (xr[k] != 0xffffffffu) {
                                const int32_t rr = r % (int32_t)BAND;
                                atomicOr((unsigned long long *)(pm + ((size_t)(r / (int32_t)BAND) * sig1 + xr[k]) * WPL + rr / 64),
                                         1ull << (rr % 64));
                            }
                        }
                        for (int32_t r0 = 64 * kRowReads; r0 < nrows; r0 += 64) {
                            // rounds with more rows than one batch of reads
                            const int32_t r = r0 + lane;
                            const uint32_t row = (uint32_t)(ell - r / (int32_t)BAND) * BAND + (uint32_t)(r % (int32_t)BAND);
                            if (r < nrows && row < m) {
                                const int32_t rr = r % (int32_t)BAND;
                                atomicOr((unsigned long long *)(pm + ((size_t)(r / (int32_t)BAND) * sig1 + xc[row]) * WPL + rr / 64),
                                         1ull << (rr % 64));
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const int32_t x = lane + 64 * k;
                            if (x < nyv) ((uint32_t *)ystage)[x] = yv[k];
                        }
                        for (int32_t x0 = 64 * 8; x0 < nyv; x0 += 64) {
                            // (uniform trip count: every lane takes part in the reads)
                            const int32_t x = x0 + lane;
                            const int32_t u = x / (int32_t)kYPerSlot;
                            const uint64_t yo = ((uint64_t)(uint32_t)__shfl((int32_t)(yoff >> 32), u & 63, 64) << 32) |
                                                (uint32_t)__shfl((int32_t)yoff, u & 63, 64);
                            const bool ok = x < nyv && __shfl(kts, u & 63, 64) >= 0;
                            if (ok) {
                                const uint16_t *ysrc = a.ystream + yo + 2 * (uint32_t)(x % (int32_t)kYPerSlot);
                                ((uint32_t *)ystage)[x] = (uint32_t)ysrc[0] | ((uint32_t)ysrc[1] << 16);
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 2; ++k) {
                            const int32_t x = lane + 64 * k;
                            if (x < ncb) cbstage[x] = cv[k];
                        }
                        for (int32_t x0 = 64 * 2; x0 < ncb; x0 += 64) {
                            const int32_t x = x0 + lane;
                            const int32_t u = x / (int32_t)(K / 32);
                            const uint64_t cb0 = ((uint64_t)(uint32_t)__shfl((int32_t)(cbo >> 32), u & 63, 64) << 32) |
                                                 (uint32_t)__shfl((int32_t)cbo, u & 63, 64);
                            const int32_t ku = __shfl(kts, u & 63, 64);
                            const uint32_t tw = (uint32_t)__shfl((int32_t)tws, u & 63, 64);
                            const uint32_t w = ((uint32_t)ku << (LOGK - 5)) + (uint32_t)(x % (int32_t)(K / 32));
                            if (x < ncb) cbstage[x] = (ku >= 0 && w < tw) ? a.cbits[cb0 + (size_t)w * 64] : 0u;
                        }
                        wave_lds_sync();
                        if (kts >= 0)
                            recompute_tile<WPL, LOGK>(tiles + (size_t)lane * SW,
                                                      pm + (size_t)(lane / NB) * sig1 * WPL,
                                                      ystage + (size_t)lane * K,
                                                      cbstage + (size_t)lane * (K / 32), V0);
                        wave_lds_sync();
                        dsl = 0;
                        khi = kt;
                        klo = kt - NB + 1 < 0 ? 0 : kt - NB + 1;
                    }
                    // walk inside the resident tiles of this band.  A window holds
                    // word q of up to 64 consecutive columns in lane registers,
                    // lane l holding column tc - l.  A diagonal step at row b of
                    // column k happens exactly when the match bit M_k[b] is set (a
                    // set match bit is the highest candidate at or below b), so a
                    // run of diagonal steps is found at once: it is the number of
                    // consecutive lanes l >= k with bit b - (l - k) of M_l set,
                    // i.e. with bit b + k of the 128-bit value M_l << l set.  The
                    // step after a run takes the top candidate bit of
                    // PM[y_j] | ~V_j at or below b.  Every bitmap word the walk
                    // passes through is written whole.
                    const int32_t rbase = ell * (int32_t)BAND;
                    const int32_t tfloor = klo << LOGK;       // first resident step
                    const uint64_t *pmd = pm + (size_t)dsl * sig1 * WPL;
                    int32_t tc = t;
                    int32_t q = (i - 1 - rbase) >> 6;
                    int32_t b = (i - 1 - rbase) & 63;
                    const int32_t wq0 = rbase >> 6;           // bitmap word of the band's word 0
                    bool leave = false;
                    while (!leave) {
                        const int32_t tl = tc - lane;
                        uint64_t VL = 0, ML = 0;
                        if (tl >= tfloor) {
                            const uint32_t sl = (uint32_t)(dsl * NB + (khi - (tl >> LOGK)));
                            const uint32_t o = (uint32_t)tl & (K - 1);
                            VL = tiles[(size_t)sl * SW + o * WPL + q];
                            const uint32_t code = (uint32_t)ystage[(size_t)sl * K + o] >> kShift;
                            ML = pmd[code * WPL + q];
                        }
                        if (wq0 + q != dwi) {
                            if (dwi >= 0 && lane == 0) dg[dwi] = dword;
                            dwi = wq0 + q;
                            dword = 0;
                        }
                        const uint64_t Slo = ML << lane;
                        const uint64_t Shi = lane ? ML >> (64 - lane) : 0ull;
                        const int32_t avail = tc - tfloor + 1;    // columns resident from tc down
                        int32_t kmax = avail < 64 ? avail : 64;
                        kmax = kmax < j ? kmax : j;
                        const uint64_t wmask = kmax >= 64 ? ~0ull : ((1ull << kmax) - 1);
                        int32_t k = 0;
                        for (;;) {
                            // diagonal run from (b, k)
                            const int32_t pl = b + k;
                            const uint64_t xs = pl < 64 ? Slo : Shi;
                            const bool bit = ((uint32_t)(xs >> (pl & 63)) & 1u) != 0;
                            const uint64_t dm = (__builtin_amdgcn_ballot_w64(bit) & wmask) >> k;
                            const int32_t run = ~dm ? (int32_t)__builtin_ctzll(~dm) : 64;
                            dword |= (run >= 64 ? ~0ull : ((1ull << run) - 1)) << (b - run + 1);
                            b -= run;
                            k += run;
                            if (b < 0 || k >= kmax) break;
                            // one general step at column k (M_k[b] is clear)
                            const uint64_t Vw = readlane64(VL, k), Mw = readlane64(ML, k);
                            const uint64_t cand = (Mw | ~Vw) & (~0ull >> (63 - b));
                            if (cand == 0) {
                                b = -1;       // climbs out of word q in column k
                                break;
                            }
                            const int32_t r = 63 - (int32_t)__builtin_clzll(cand);
                            const uint32_t d = (uint32_t)(Mw >> r) & 1u;
                            dword |= (uint64_t)d << r;
                            b = r - (int32_t)d;
                            ++k;
                            if (b < 0 || k >= kmax) break;
                        }
                        j -= k;
                        tc -= k;
                        if (b < 0) {
                            // on to row 63 of word q-1 in column j, or out of the band
                            if (q == 0) {
                                leave = true;
                            } else {
                                if (lane == 0) dg[dwi] = dword;
                                --q;
                                --dwi;
                                dword = 0;
                                b = 63;
                            }
                        }
                        if (j == 0 || tc < tfloor) leave = true;
                    }
                    i = rbase + q * 64 + b + 1;
                    if (i == rbase) {
                        // left band ell through its bottom row
                        if (lane == 0) dg[dwi] = dword;
                        dwi = -1;
                        dword = 0;
                        if (rec && lane == 0) cross[ell] = (uint32_t)j;
                        if (cmp && (int32_t)cross[ell] == j) {
                            merged = true;
                            break;
                        }
                    }
                }
                if (!merged) {
                    if (dwi >= 0 && lane == 0) dg[dwi] = dword;
                    if (j == 0 && i > i_stop) {
                        // the walk ended inside the strip: rows i_stop+1..i
                        // take no diagonal step
                        if (rec)
                            for (int32_t g = i_stop / (int32_t)BAND + lane; g <= (i - 1) / (int32_t)BAND;
                                 g += 64)
                                cross[g] = 0;
                        if (!rec)
                            for (int32_t w = i_stop / 64 + lane; w < i / 64; w += 64) dg[w] = 0;
                    }
                }
            }
            if (a.mode == kTbFix) {
                if (lane == 0) {
                    sres[2 * s] = (uint32_t)e;
                    sres[2 * s + 1] = (!walk || merged) ? cross[s * G] : (uint32_t)j;
                }
            } else if (a.mode == kTbSeal) {
                e = walk ? j : (int32_t)sres[2 * s + 1];
            }
            if (a.mode != kTbSeal || s == 0) break;
            --s;
        }
    }
}

// The bitmap of diagonal rows, read in row order, selects the symbols of X
// that form the LCS.  One wave per item of 64 bitmap words of a pair: the
// item's output starts at the number of set bits in the words before it;
// each lane places the symbols of its word in an LDS staging buffer at its
// prefix-sum offset, and the wave then writes the buffer out with
// consecutive lanes on consecutive bytes.  The item holding a pair's last
// word checks the pair's total against its length.
__global__ __launch_bounds__(256) void k_emit(EmitArgs a) {
    __shared__ uint8_t stage_all[4][64 * 64];
    const int lane = threadIdx.x & 63;
    uint8_t *stage = stage_all[threadIdx.x >> 6];
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t it = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); it < a.nitems;
         it += waves) {
        const uint32_t p = a.em_pair[it];
        const uint32_t w0 = a.em_w0[it];
        const uint32_t m = a.pair_m[p];
        const uint32_t n = a.pair_n[p];
        const uint64_t cap = m < n ? m : n;     // the pair's slot in `out`
        const uint32_t W = (m + 63) / 64;
        const uint64_t *bm = a.diag + a.pair_diag[p];
        const uint8_t *x = a.xbytes + a.pair_xoff[p];
        uint8_t *o = a.out + a.pair_out[p];
        uint32_t before = 0;
        for (uint32_t v = lane; v < w0; v += 64) before += (uint32_t)__builtin_popcountll(bm[v]);
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) before += __shfl_xor(before, d, 64);
        const uint32_t w = w0 + lane;
        uint64_t bits = 0;
        uint4 xv[4] = {};
        if (w < W) {
            // the word's 64 symbols at once (X is padded to whole words)
            bits = bm[w];
            const uint4 *xs = (const uint4 *)(x + (size_t)w * 64);
#pragma unroll
            for (int k = 0; k < 4; ++k) xv[k] = xs[k];
        }
        const uint32_t c = (uint32_t)__builtin_popcountll(bits);
        uint32_t incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t up = __shfl_up(incl, d, 64);
            if (lane >= d) incl += up;
        }
        const uint32_t total = __shfl(incl, 63, 64);
        uint32_t pos = incl - c;
        const uint32_t xw[16] = {xv[0].x, xv[0].y, xv[0].z, xv[0].w, xv[1].x, xv[1].y,
                                 xv[1].z, xv[1].w, xv[2].x, xv[2].y, xv[2].z, xv[2].w,
                                 xv[3].x, xv[3].y, xv[3].z, xv[3].w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            // rows 4k+1 .. 4k+4 of the word
            uint32_t mk = (uint32_t)(bits >> (4 * k)) & 0xfu;
            while (mk) {
                const int r = __builtin_ctz(mk);
                stage[pos++] = (uint8_t)(xw[k] >> (8 * r));
                mk &= mk - 1;
            }
        }
        wave_lds_sync();
        const uint64_t base = before;
        for (uint32_t e = lane; e < total; e += 64)
            if (base + e < cap) o[base + e] = stage[e];
        wave_lds_sync();
        if (lane == 0 && w0 + 64 >= W && base + total != a.out_len[p]) atomicOr(a.error, 2u);
    }
}

hipError_t launch_emit(const EmitArgs &a, hipStream_t s) {
    if (!a.nitems) return hipSuccess;
    uint32_t blocks = (a.nitems + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_emit, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

#define LCS_TB_SYM(W)                                              \
    (logk == 6 ? (const void *)&k_traceback<W, 6>                  \
               : logk == 7 ? (const void *)&k_traceback<W, 7>      \
                           : (const void *)&k_traceback<W, 8>)
const void *tb_symbol(int wpl, int ckpt_every) {
    const int logk = ckpt_every == 64 ? 6 : ckpt_every == 128 ? 7 : 8;
    switch (wpl) {
        case 1: return LCS_TB_SYM(1);
        case 2: return LCS_TB_SYM(2);
        case 4: return LCS_TB_SYM(4);
        default: return LCS_TB_SYM(8);
    }
}
#undef LCS_TB_SYM

hipError_t launch_tb(int wpl, const TbArgs &a, uint32_t grid, hipStream_t s) {
    if (a.ckpt_every != 64 && a.ckpt_every != 128 && a.ckpt_every != 256) return hipErrorInvalidValue;
    const size_t lds = tb_lds_bytes(wpl, a.sigma, a.ckpt_every, a.nb, a.nbands);
    const int logk = a.ckpt_every == 64 ? 6 : a.ckpt_every == 128 ? 7 : 8;
#define LCS_TB_LAUNCH(W, L)                                                               \
    if (wpl == W && logk == L) {                                                          \
        hipLaunchKernelGGL((k_traceback<W, L>), dim3(grid), dim3(kTbBlock), lds, s, a); \
        return hipGetLastError();                                                         \
    }
    LCS_TB_LAUNCH(1, 6) LCS_TB_LAUNCH(1, 7) LCS_TB_LAUNCH(1, 8)
    LCS_TB_LAUNCH(2, 6) LCS_TB_LAUNCH(2, 7) LCS_TB_LAUNCH(2, 8)
    LCS_TB_LAUNCH(4, 6) LCS_TB_LAUNCH(4, 7) LCS_TB_LAUNCH(4, 8)
    LCS_TB_LAUNCH(8, 6) LCS_TB_LAUNCH(8, 7) LCS_TB_LAUNCH(8, 8)
#undef LCS_TB_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace lcs
