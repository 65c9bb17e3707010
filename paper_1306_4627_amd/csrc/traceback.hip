// traceback.hip -- the canonical traceback and the emit of the LCS bytes.
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
#include "bitvec.hpp"
#include "plan.hpp"

namespace lcs {

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

size_t tb_lds_bytes(int wpl, int sigma, int K, int nb, int bands, int waves) {
    return (size_t)waves * tb_wave_words(wpl, sigma, K, nb, bands) * sizeof(uint64_t);
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
                                               const uint32_t *cbs, const uint64_t (&V0)[WPL],
                                               uint32_t ysh) {
    constexpr uint32_t K = 1u << LOGK;
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
                const uint32_t code = ((k & 1) ? (yw[k >> 1] >> 16) : (yw[k >> 1] & 0xffffu)) >> ysh;
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
    const uint32_t ysh = (uint32_t)a.ysh;   // stream value -> symbol code
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
        // the seal pass runs down a group of strips: the pair's strips, or in
        // traceback rounds the strips of one round
        const bool seal = a.mode == kTbSeal;
        const int32_t s_top = seal && a.tk_s ? (int32_t)a.tk_s[ticket] : S - 1;
        const int32_t s_lo = seal && a.tk_lo ? (int32_t)a.tk_lo[ticket] : 0;
        const bool from_above = !seal && (a.tk_s[ticket] & kFromAbove) != 0;
        int32_t s = seal ? s_top - 1 : (int32_t)(a.tk_s[ticket] & ~kFromAbove);
        // seal: exit column of the strip above the current one
        int32_t e = seal ? (int32_t)cross[s_top * G] : 0;

        for (;;) {
            const int32_t top = (s + 1) * R;       // first row above strip s
            // column at which the speculative walk enters strip s
            const uint32_t guess_raw = (uint32_t)(((uint64_t)(uint32_t)top * n) / m);
            const int32_t guess = guess_raw < 1u ? 1 : (int32_t)guess_raw;
            int32_t i = top, j = 0;
            bool walk = true;
            // every pass records the columns where its walk leaves each band,
            // so `cross` always describes the path now in the bitmap; the
            // fix-up and seal passes stop where their walk meets that path
            // (from the same position the walks coincide)
            const bool cmp = a.mode != kTbSpec;
            if (a.mode == kTbSpec) {
                if (s == S - 1) {
                    i = (int32_t)m;
                    j = (int32_t)n;
                } else if (from_above) {
                    // the path above this strip is final (an earlier round)
                    j = (int32_t)cross[(s + 1) * G];
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
                                                      cbstage + (size_t)lane * (K / 32), V0, ysh);
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
                            const uint32_t code = (uint32_t)ystage[(size_t)sl * K + o] >> ysh;
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
                        if (cmp && (int32_t)cross[ell] == j) {
                            merged = true;
                            break;
                        }
                        if (lane == 0) cross[ell] = (uint32_t)j;
                    }
                }
                if (!merged) {
                    if (dwi >= 0 && lane == 0) dg[dwi] = dword;
                    if (j == 0 && i > i_stop) {
                        // the walk ended inside the strip: rows i_stop+1..i
                        // take no diagonal step
                        for (int32_t g = i_stop / (int32_t)BAND + lane; g <= (i - 1) / (int32_t)BAND;
                             g += 64)
                            cross[g] = 0;
                        if (cmp)
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
                // a walk that met the recorded path leaves the strip where
                // that path does
                e = !walk ? (int32_t)sres[2 * s + 1] : merged ? (int32_t)cross[s * G] : j;
            }
            if (a.mode != kTbSeal || s == s_lo) break;
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

hipError_t launch_tb(int wpl, const TbArgs &a, uint32_t grid, int waves, hipStream_t s) {
    if (a.ckpt_every != 64 && a.ckpt_every != 128 && a.ckpt_every != 256) return hipErrorInvalidValue;
    if (waves < 1 || waves > kTbBlock / 64) return hipErrorInvalidValue;
    const size_t lds = tb_lds_bytes(wpl, a.sigma, a.ckpt_every, a.nb, a.nbands, waves);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int logk = a.ckpt_every == 64 ? 6 : a.ckpt_every == 128 ? 7 : 8;
#define LCS_TB_LAUNCH(W, L)                                                               \
    if (wpl == W && logk == L) {                                                          \
        hipLaunchKernelGGL((k_traceback<W, L>), dim3(grid), dim3(64 * waves), lds, s, a); \
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
