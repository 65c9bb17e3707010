// bitvec.hpp -- device helpers shared by the fill and the traceback kernels.
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

#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lcs {

// One column step for WPL words of one lane: U = V & M, S = V + U + carry
// (64*WPL-bit add, carry in and out as a wave lane mask in an SGPR pair),
// V' = S | (V & ~M).  Six VALU instructions per 64 cells.
//
// The carry mask is written by a VALU instruction (v_addc_co_u32) and read
// by the next v_addc_co_u32; gfx950 needs two wait states between the two,
// which the order below provides with independent instructions: inside a
// word the low-half bitop3 and the high-half AND sit between the two adds;
// across words the high-half bitop3 of the previous word and the low-half
// AND of the next one do.  The compiler cannot see into an asm statement and
// pads every boundary between two of them that pass the mask with a wait
// state, so words go two to a statement.  In the fill the carry mask coming
// in is written by scalar instructions and the one going out is only read by
// scalar instructions, which need no wait states; a caller that writes the
// mask coming in with a VALU instruction puts two wait states after it.
template <int WPL>
__device__ __forceinline__ void column_step(uint32_t (&vlo)[WPL], uint32_t (&vhi)[WPL],
                                            const uint64_t (&M)[WPL], uint64_t &carry) {
    if constexpr (WPL == 1) {
        const uint32_t mlo = (uint32_t)M[0], mhi = (uint32_t)(M[0] >> 32);
        uint32_t t0, t1;
        asm("v_and_b32 %[ulo], %[vlo], %[mlo]\n\t"
            "v_addc_co_u32 %[ulo], %[c], %[vlo], %[ulo], %[c]\n\t"
            "v_bitop3_b32 %[vlo], %[ulo], %[vlo], %[mlo] bitop3:0xf4\n\t"
            "v_and_b32 %[uhi], %[vhi], %[mhi]\n\t"
            "v_addc_co_u32 %[uhi], %[c], %[vhi], %[uhi], %[c]\n\t"
            "v_bitop3_b32 %[vhi], %[uhi], %[vhi], %[mhi] bitop3:0xf4"
            : [vlo] "+v"(vlo[0]), [vhi] "+v"(vhi[0]), [c] "+s"(carry), [ulo] "=&v"(t0),
              [uhi] "=&v"(t1)
            : [mlo] "v"(mlo), [mhi] "v"(mhi));
    } else {
#pragma unroll
        for (int q = 0; q < WPL; q += 2) {
            const uint32_t mlo0 = (uint32_t)M[q], mhi0 = (uint32_t)(M[q] >> 32);
            const uint32_t mlo1 = (uint32_t)M[q + 1], mhi1 = (uint32_t)(M[q + 1] >> 32);
            uint32_t t0, t1;
            asm("v_and_b32 %[ulo], %[vlo0], %[mlo0]\n\t"
                "v_addc_co_u32 %[ulo], %[c], %[vlo0], %[ulo], %[c]\n\t"
                "v_bitop3_b32 %[vlo0], %[ulo], %[vlo0], %[mlo0] bitop3:0xf4\n\t"
                "v_and_b32 %[uhi], %[vhi0], %[mhi0]\n\t"
                "v_addc_co_u32 %[uhi], %[c], %[vhi0], %[uhi], %[c]\n\t"
                "v_bitop3_b32 %[vhi0], %[uhi], %[vhi0], %[mhi0] bitop3:0xf4\n\t"
                "v_and_b32 %[ulo], %[vlo1], %[mlo1]\n\t"
                "v_addc_co_u32 %[ulo], %[c], %[vlo1], %[ulo], %[c]\n\t"
                "v_bitop3_b32 %[vlo1], %[ulo], %[vlo1], %[mlo1] bitop3:0xf4\n\t"
                "v_and_b32 %[uhi], %[vhi1], %[mhi1]\n\t"
                "v_addc_co_u32 %[uhi], %[c], %[vhi1], %[uhi], %[c]\n\t"
                "v_bitop3_b32 %[vhi1], %[uhi], %[vhi1], %[mhi1] bitop3:0xf4"
                : [vlo0] "+v"(vlo[q]), [vhi0] "+v"(vhi[q]), [vlo1] "+v"(vlo[q + 1]),
                  [vhi1] "+v"(vhi[q + 1]), [c] "+s"(carry), [ulo] "=&v"(t0), [uhi] "=&v"(t1)
                : [mlo0] "v"(mlo0), [mhi0] "v"(mhi0), [mlo1] "v"(mlo1), [mhi1] "v"(mhi1));
        }
    }
}

// Make a value the compiler cannot prove wave-uniform live in SGPRs again (a
// no-op when it already does).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
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

}  // namespace lcs
