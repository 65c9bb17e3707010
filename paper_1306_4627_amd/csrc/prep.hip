// prep.hip -- per-pass input preparation: symbol remap of X, the zeroed
// scratch words (and the starting state of a threshold pass), and the
// per-segment Y streams read by the fill.
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

}  // namespace lcs
