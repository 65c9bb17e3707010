// prep.hip -- per-pass input preparation: symbol remap of X, the zeroed
// scratch words (and the starting state of a threshold pass), and the
// per-segment Y streams read by the fill.
#include "kernels.hpp"

namespace lcs {

// --------------------------------------------------------------------------
// prep: symbol remap (bytes -> codes), Y streams, zeroing -- one launch
// --------------------------------------------------------------------------

// The work-groups of the one prep launch split into three ranges: the X
// remap (and the reversed X of split pairs), the zeroing and the Y streams.
// All three only depend on the batch's inputs, so they run side by side.
struct PrepSplit {
    uint32_t remap_end, zero_end, total;
};

static PrepSplit prep_split(const PrepArgs &a, uint64_t xbytes_n) {
    PrepSplit p{};
    uint64_t rb = (xbytes_n / 16 + 255) / 256;
    if (rb > 4096) rb = 4096;
    const uint64_t zw = a.npairs + a.nzero + a.nzero64;
    uint64_t zb = (zw + 255) / 256;
    if (zb > 1024) zb = 1024;
    if (zb < 1) zb = 1;
    uint64_t sb = (a.nblk * 2 + 255) / 256;
    if (sb > 16384) sb = 16384;
    p.remap_end = (uint32_t)rb;
    p.zero_end = (uint32_t)(rb + zb);
    p.total = (uint32_t)(rb + zb + sb);
    return p;
}

// Symbol remap of the X arena, sixteen bytes per thread (both arenas start
// 256-byte aligned), the byte -> code table in LDS.
__device__ __forceinline__ void remap_x(const uint8_t *lut, const uint8_t *__restrict__ src,
                                        uint8_t *__restrict__ dst, uint64_t n, uint32_t block,
                                        uint32_t blocks) {
    const auto map4 = [&](uint32_t w) {
        return (uint32_t)lut[w & 0xff] | ((uint32_t)lut[(w >> 8) & 0xff] << 8) |
               ((uint32_t)lut[(w >> 16) & 0xff] << 16) | ((uint32_t)lut[w >> 24] << 24);
    };
    const uint64_t stride = (uint64_t)blocks * blockDim.x * 16;
    for (uint64_t i = ((uint64_t)block * blockDim.x + threadIdx.x) * 16; i < n; i += stride) {
        if (i + 16 <= n) {
            const uint4 w = *(const uint4 *)(src + i);
            uint4 r;
            r.x = map4(w.x);
            r.y = map4(w.y);
            r.z = map4(w.z);
            r.w = map4(w.w);
            *(uint4 *)(dst + i) = r;
        } else {
            for (uint64_t k = i; k < n; ++k) dst[k] = lut[src[k]];
        }
    }
}

__device__ __forceinline__ void zero_words(const PrepArgs &a, uint32_t block, uint32_t blocks) {
    const uint64_t tid = (uint64_t)block * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)blocks * blockDim.x;
    for (uint64_t k = tid; k < a.npairs; k += stride) a.out_len[k] = 0;
    for (uint64_t k = tid; k < a.nzero; k += stride) a.zero_words[k] = 0;
    for (uint64_t k = tid; k < a.nzero64; k += stride) a.zero64[k] = 0;
    // threshold pass: a target of 0 is reached before any column, and no
    // pair can reach one above min(m, n) (the length never exceeds either)
    if (a.thr_dec)
        for (uint64_t k = tid; k < a.npairs; k += stride) {
            const uint32_t T = a.thr_t[k], m = a.pair_m[k], n = a.pair_n[k];
            a.thr_dec[k] = T == 0 ? 1u : (T > (m < n ? m : n) ? 2u : 0u);
        }
}

// Reversed codes of the X of every split pair (one byte per thread, the
// rows past m of the last 64 set to code 0: the fill masks them out).  Each
// copy starts 64-byte aligned in the X-code arena past the remapped range,
// so the remap and these writes never meet.
__device__ __forceinline__ void reverse_x(const uint8_t *lut, const PrepArgs &a, uint32_t block,
                                          uint32_t blocks) {
    const uint64_t tid = (uint64_t)block * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)blocks * blockDim.x;
    for (uint32_t s = 0; s < a.nhalves; ++s) {
        const HalfInfo h = a.halves[s];
        const uint64_t padded = ((uint64_t)h.m + 63) / 64 * 64;
        for (uint64_t r = tid; r < padded; r += stride)
            a.xcodes[h.xdst + r] = r < h.m ? lut[a.xbytes[h.xsrc + h.m - 1 - r]] : (uint8_t)0;
    }
}

// Eight stream values of a region from element kg on: codes of Y at columns
// 0..n-1 (with `rev`, column c holds Y[n-1-c]), the sentinel code everywhere
// else, each shifted into a byte offset of its row of match masks; two per
// 32-bit word.
__device__ __forceinline__ uint4 stream8(const uint8_t *lut, const uint8_t *y, uint64_t kg,
                                         uint32_t pre, uint32_t n, uint32_t sh, uint32_t sent,
                                         bool rev) {
    uint32_t c[8];
    if (kg >= pre && kg + 8 <= (uint64_t)pre + n) {
        // eight bytes of Y from two aligned 8-byte reads (the Y arena is
        // padded by 64 bytes); reversed, the eight bytes ending at column
        // n-1-(kg-pre), byte-swapped
        const uint64_t c0 = kg - pre;
        const uintptr_t ad = (uintptr_t)(y + (rev ? n - 8 - c0 : c0));
        const uint64_t *al = (const uint64_t *)(ad & ~(uintptr_t)7);
        const uint32_t s8 = (uint32_t)(ad & 7) * 8;
        const uint64_t lo = al[0], hi = al[1];
        uint64_t v = s8 ? (lo >> s8) | (hi << (64 - s8)) : lo;
        if (rev) v = __builtin_bswap64(v);
#pragma unroll
        for (int e = 0; e < 8; ++e) c[e] = (uint32_t)lut[(uint32_t)(v >> (8 * e)) & 0xffu] << sh;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint64_t k = kg + e;
            const uint64_t col = k - pre;
            c[e] = (k >= pre && col < n) ? ((uint32_t)lut[y[rev ? n - 1 - col : col]] << sh) : sent;
        }
    }
    uint4 v;
    v.x = c[0] | (c[1] << 16);
    v.y = c[2] | (c[3] << 16);
    v.z = c[4] | (c[5] << 16);
    v.w = c[6] | (c[7] << 16);
    return v;
}

// One thread per 32 stream elements (grid-stride over the stream's 64-element
// blocks, two threads a block): the region of every block comes from a
// table, its description from one 32-byte record, so a batch of many short
// regions costs no more threads than one of a few long ones.
__device__ __forceinline__ void streams(const PrepArgs &a, const uint8_t *lut, uint32_t block,
                                        uint32_t blocks) {
    const uint64_t halves = a.nblk * 2;
    const uint64_t stride = (uint64_t)blocks * blockDim.x;
    for (uint64_t h = (uint64_t)block * blockDim.x + threadIdx.x; h < halves; h += stride) {
        const SegInfo &sg = a.seg[a.blk_seg[h >> 1]];
        const uint4 m0 = *(const uint4 *)&sg;              // begin, yoff
        const uint4 m1 = *((const uint4 *)&sg + 1);        // len, pre, n, shift
        const uint64_t begin = ((uint64_t)m0.y << 32) | m0.x;
        const uint64_t yoff = ((uint64_t)m0.w << 32) | m0.z;
        const uint64_t k0 = h * 32 - begin;   // element offset in the region
        if (k0 >= m1.x) continue;             // padding to the block
        const uint8_t *y = a.ybytes + yoff;
        const uint32_t sh = m1.w & (kSegReversed - 1);
        const bool rev = (m1.w & kSegReversed) != 0;
        const uint32_t sent = (uint32_t)a.sentinel << sh;
        uint4 v[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) v[g] = stream8(lut, y, k0 + 8 * g, m1.y, m1.z, sh, sent, rev);
        uint4 *dst = (uint4 *)(a.ystream + h * 32);
#pragma unroll
        for (int g = 0; g < 4; ++g)
            if (k0 + 8 * g < m1.x) dst[g] = v[g];
    }
}

__global__ __launch_bounds__(256) void k_prep(PrepArgs a, uint64_t xbytes_n, PrepSplit sp) {
    __shared__ uint8_t lut[256];
    lut[threadIdx.x] = a.lut[threadIdx.x];
    __syncthreads();
    const uint32_t b = blockIdx.x;
    if (b < sp.remap_end) {
        remap_x(lut, a.xbytes, a.xcodes, xbytes_n, b, sp.remap_end);
        if (a.nhalves) reverse_x(lut, a, b, sp.remap_end);
    } else if (b < sp.zero_end) {
        zero_words(a, b - sp.remap_end, sp.zero_end - sp.remap_end);
    } else {
        streams(a, lut, b - sp.zero_end, sp.total - sp.zero_end);
    }
}

hipError_t launch_prep(const PrepArgs &a, uint64_t xbytes_n, hipStream_t s) {
    const PrepSplit sp = prep_split(a, xbytes_n);
    hipLaunchKernelGGL(k_prep, dim3(sp.total), dim3(256), 0, s, a, xbytes_n, sp);
    return hipGetLastError();
}

}  // namespace lcs
