// halves.hip -- the length of a pair from two fills of half its columns.
//
// Cut section I.C's table at column h.  Every path from (0, 0) to (m, n)
// crosses column h, so c[m][n] is the largest, over the rows k, of c[k][h]
// (X[1..k] against Y[1..h]) plus the LCS of X[k+1..m] with Y[h+1..n] -- the
// middle-column split Hirschberg's method is built on.  The fill runs the two
// halves side by side: X against Y[1..h], and X reversed against Y[h+1..n]
// reversed, whose table at row m - k holds that second term.  Both store
// their last column V (bit i clear exactly when the column steps up at row
// i + 1), so with
//   f_i = 1 - bit i of V_first            (c[i+1][h] - c[i][h])
//   g_i = 1 - bit (m-1-i) of V_second     (the second term loses row i+1)
// the sum at row k is D(k) = sum_{i<k} f_i + sum_{i>=k} g_i, and
//   c[m][n] = max_k D(k) = G + max(0, max_k sum_{i<k} (f_i - g_i)),  G = sum_i g_i.
#include "kernels.hpp"

namespace lcs {

constexpr int kHalvesBlock = 1024;

// `cnt` (1..64) bits of a bit string from bit s on, as the low bits of a word.
__device__ __forceinline__ uint64_t bit_window(const uint64_t *v, uint64_t s, uint32_t cnt) {
    const uint64_t w = s >> 6;
    const uint32_t o = (uint32_t)(s & 63);
    uint64_t r = v[w] >> o;
    if (o && o + cnt > 64) r |= v[w + 1] << (64 - o);
    return cnt == 64 ? r : r & ((1ull << cnt) - 1);
}

// One work-group per split pair.  Each thread takes a run of consecutive
// 64-row words and reduces it to (sum, best prefix) of f - g, the empty
// prefix included, four rows at a time: a 256-entry table gives, for the four
// rows' up bits (f and not g) and down bits (g and not f), their sum and best
// prefix.  The runs are then joined in row order by a tree of the
// (associative) join (s1, b1).(s2, b2) = (s1 + s2, max(b1, s1 + b2)).
__global__ __launch_bounds__(kHalvesBlock) void k_halves(HalvesArgs a) {
    __shared__ int32_t s_sum[kHalvesBlock], s_best[kHalvesBlock];
    __shared__ uint32_t s_g[kHalvesBlock];
    __shared__ uint8_t s_tab[256];   // best | (sum + 4) << 4 of four rows
    const uint32_t tid = threadIdx.x;
    if (tid < 256) {
        int32_t sm = 0, bs = 0;
        for (int i = 0; i < 4; ++i) {
            sm += (int32_t)((tid >> (4 + i)) & 1u) - (int32_t)((tid >> i) & 1u);
            bs = sm > bs ? sm : bs;
        }
        s_tab[tid] = (uint8_t)(bs | ((sm + 4) << 4));
    }
    __syncthreads();
    const HalfInfo h = a.halves[blockIdx.x];
    const uint32_t m = h.m;
    const uint32_t W = (m + 63) / 64;
    const uint64_t *vf = a.v + h.vf;
    const uint64_t *vb = a.v + h.vb;
    const uint32_t per = (W + kHalvesBlock - 1) / kHalvesBlock;
    const uint32_t w0 = min(W, tid * per), w1 = min(W, w0 + per);
    int32_t sum = 0, best = 0;
    uint32_t gsum = 0;
    for (uint32_t w = w0; w < w1; ++w) {
        const uint32_t row0 = w * 64;
        const uint32_t cnt = min(64u, m - row0);
        const uint64_t valid = cnt == 64 ? ~0ull : (1ull << cnt) - 1;
        const uint64_t f = ~vf[w] & valid;
        // rows row0 .. row0+cnt-1 are rows m-1-row0 down to m-row0-cnt of
        // the reversed half: that window, bit order reversed
        const uint64_t win = bit_window(vb, (uint64_t)(m - row0 - cnt), cnt);
        const uint64_t g = ~(__builtin_bitreverse64(win) >> (64 - cnt)) & valid;
        gsum += (uint32_t)__builtin_popcountll(g);
        const uint64_t up = f & ~g, down = g & ~f;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t e = s_tab[(((uint32_t)(up >> (4 * q)) & 15u) << 4) |
                                     ((uint32_t)(down >> (4 * q)) & 15u)];
            const int32_t b4 = sum + (int32_t)(e & 15u);
            best = b4 > best ? b4 : best;
            sum += (int32_t)(e >> 4) - 4;
        }
    }
    s_sum[tid] = sum;
    s_best[tid] = best;
    s_g[tid] = gsum;
    for (uint32_t st = 1; st < kHalvesBlock; st *= 2) {
        __syncthreads();
        if ((tid & (2 * st - 1)) == 0) {
            const int32_t b2 = s_sum[tid] + s_best[tid + st];
            s_best[tid] = b2 > s_best[tid] ? b2 : s_best[tid];
            s_sum[tid] += s_sum[tid + st];
            s_g[tid] += s_g[tid + st];
        }
    }
    __syncthreads();
    if (tid == 0) a.out_len[h.pair] = (uint64_t)s_g[0] + (uint64_t)s_best[0];
}

hipError_t launch_halves(const HalvesArgs &a, hipStream_t s) {
    if (!a.nhalves) return hipSuccess;
    hipLaunchKernelGGL(k_halves, dim3(a.nhalves), dim3(kHalvesBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace lcs
