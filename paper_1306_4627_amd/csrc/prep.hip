// prep.hip -- per-pass input preparation: symbol remap of X, the zeroed
// scratch words (and the starting state of a threshold pass), and the
// per-segment Y streams read by the fill.
#include "kernels.hpp"

namespace lcs {

// --------------------------------------------------------------------------
// prep: symbol remap (bytes -> codes), Y streams, zeroing
// --------------------------------------------------------------------------

// Symbol remap of the X arena, sixteen bytes per thread (both arenas start
// 256-byte aligned), the byte -> code table in LDS.
__global__ __launch_bounds__(256) void k_remap_x(const uint8_t *__restrict__ lut_g,
                                                 const uint8_t *__restrict__ src,
                                                 uint8_t *__restrict__ dst, uint64_t n) {
    __shared__ uint8_t lut[256];
    lut[threadIdx.x] = lut_g[threadIdx.x];
    __syncthreads();
    const auto map4 = [&](uint32_t w) {
        return (uint32_t)lut[w & 0xff] | ((uint32_t)lut[(w >> 8) & 0xff] << 8) |
               ((uint32_t)lut[(w >> 16) & 0xff] << 16) | ((uint32_t)lut[w >> 24] << 24);
    };
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 16;
    for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16; i < n; i += stride) {
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

// One thread per sixteen stream elements over the whole stream (grid-stride):
// codes of Y at columns 0..n-1 of each region, the sentinel code everywhere
// else in it, each shifted into a byte offset of its row of match masks.
// The region of every 64-element block comes from a table, so a batch of
// many short regions costs no more work-groups than one of a few long ones.
__global__ __launch_bounds__(256) void k_streams(PrepArgs a) {
    // the byte -> code table in LDS; each thread writes two groups of eight
    // stream values (16 bytes each, aligned: regions start at multiples of 64
    // elements)
    __shared__ uint8_t lut[256];
    lut[threadIdx.x] = a.lut[threadIdx.x];
    __syncthreads();
    const uint64_t halves = a.nblk * 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < halves; h += stride) {
        const uint32_t s = a.blk_seg[h >> 2];
        const uint64_t k0 = h * 16 - a.seg_begin[s];  // element offset in the region
        const uint64_t len = a.seg_len[s];
        if (k0 >= len) continue;                      // padding to the block
        const uint64_t pre = a.seg_pre[s];
        const uint64_t n = a.seg_n[s];
        const uint32_t sh = a.seg_shift[s];
        const uint8_t *y = a.ybytes + a.seg_yoff[s];
        const uint32_t sent = (uint32_t)a.sentinel << sh;
        const auto group = [&](uint64_t kg) {
            uint32_t c[8];
            if (kg >= pre && kg + 8 <= pre + n) {
                // eight bytes of Y from two aligned 8-byte reads (the Y arena
                // is padded by 64 bytes)
                const uintptr_t ad = (uintptr_t)(y + (kg - pre));
                const uint64_t *al = (const uint64_t *)(ad & ~(uintptr_t)7);
                const uint32_t s8 = (uint32_t)(ad & 7) * 8;
                const uint64_t lo = al[0], hi = al[1];
                const uint64_t v = s8 ? (lo >> s8) | (hi << (64 - s8)) : lo;
#pragma unroll
                for (int e = 0; e < 8; ++e) c[e] = (uint32_t)(v >> (8 * e)) & 0xffu;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint64_t k = kg + e;
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
            return v;
        };
        const uint4 v0 = group(k0);
        if (k0 + 8 < len) {
            const uint4 v1 = group(k0 + 8);
            *(uint4 *)(a.ystream + h * 16) = v0;
            *(uint4 *)(a.ystream + h * 16 + 8) = v1;
        } else {
            *(uint4 *)(a.ystream + h * 16) = v0;
        }
    }
}

__global__ void k_zero(PrepArgs a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
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

hipError_t launch_prep(const PrepArgs &a, uint64_t xbytes_n, hipStream_t s) {
    if (xbytes_n) {
        uint64_t blocks = (xbytes_n / 16 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_remap_x, dim3((uint32_t)blocks), dim3(256), 0, s, a.lut, a.xbytes,
                           a.xcodes, xbytes_n);
    }
    hipLaunchKernelGGL(k_zero, dim3(512), dim3(256), 0, s, a);
    if (a.nblk) {
        uint64_t blocks = (a.nblk * 4 + 255) / 256;
        if (blocks > 32768) blocks = 32768;
        hipLaunchKernelGGL(k_streams, dim3((uint32_t)blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace lcs
