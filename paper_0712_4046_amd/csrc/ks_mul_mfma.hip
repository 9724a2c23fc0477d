// ks_mul_mfma.hip -- integer products on the int8 matrix cores (v_mfma_i32_32x32x32_i8).
//
// An integer product is a convolution of digit sequences: with 7-bit digits a_i, b_j
// (values 0..127, so they fit the signed int8 operands exactly and no sign correction is
// needed), C[k] = sum_i a_i b_{k-i} and A*B = sum_k C[k] 2^(7k).  Writing k = 32 s + r and
// splitting the shift into 32-digit blocks t,
//     C[32 s + r] = sum_t sum_{q<32} a[32 (s - t) + q] * b[32 t + r - q],
// each block shift t is a 32x32x32 matrix product: rows s (a 32-digit output block), columns
// r, contraction q; the a-matrix rows are contiguous 32-digit runs of a and the b-matrix is a
// Toeplitz tile of b.  One v_mfma_i32_32x32x32_i8 computes it, accumulating exactly in int32
// (at most 32 * 127^2 per step, so up to MFMA_MAX_STEPS steps per accumulator).
//
// Lane layout of v_mfma_i32_32x32x32_i8 (checked on the device): lane l supplies row (A) or
// column (B) l % 32 and contraction indices 16 (l / 32) .. + 15 as 16 bytes; result register
// i of lane l is row 8 (i / 4) + 4 (l / 32) + (i % 4), column l % 32.
//
// A block covers MFMA_RT row tiles (32 rows each, so 32 * 32 * MFMA_RT output digits =
// MFMA_LIMBS limbs) and its MFMA_WAVES waves split the block's range of t between them.  Each
// wave stages its digit windows through LDS (the b window is read back at per-lane byte
// offsets and realigned with v_alignbyte).  At the end the waves add their column sums into
// LDS limb accumulators, and the block writes the same three-piece columns as the vector-ALU
// multiplier, so the recombination stage is shared.
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---- digits ------------------------------------------------------------------------------------

// out[x] for x in [0, len): digit d = (reversed ? base - x : x - base) of the limb array, where
// digit d is bits [7 d, 7 d + 7) for 0 <= d < nd and 0 otherwise.  Four bytes per thread.
__global__ __launch_bounds__(256) void digitize_kernel(Launch<DigitJob> L) {
    int64_t local;
    const DigitJob J = get_job(L, (int64_t)blockIdx.x, local);
    const int64_t x0 = (local * 256 + threadIdx.x) * 4;
    if (x0 >= J.len) return;
    uint32_t word = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t x = x0 + b;
        const int64_t d = J.reversed ? J.base - x : x - J.base;
        uint32_t v = 0;
        if (d >= 0 && d < J.nd) v = bits_word(J.limbs, J.n, 7 * d) & 0x7fu;
        word |= v << (8 * b);
    }
    *reinterpret_cast<uint32_t *>(J.out + x0) = word;
}

// ---- products ----------------------------------------------------------------------------------

__global__ __launch_bounds__(MFMA_TPB) void mul_mfma_kernel(Launch<MfmaJob> L) {
    // per wave: a window (32 (MFMA_ROWS + MFMA_TC) bytes) and b window (32 MFMA_TC + 64 bytes)
    constexpr int AWIN = 32 * (MFMA_ROWS + MFMA_TC);
    constexpr int BWIN = 32 * MFMA_TC + 64;
    constexpr int WBYTES = AWIN + BWIN;
    __shared__ __attribute__((aligned(16))) uint8_t lds[MFMA_WAVES * WBYTES];
    static_assert(MFMA_WAVES * WBYTES >= 2 * MFMA_LIMBS * 8, "LDS too small for the reduction");

    int64_t local;
    const MfmaJob J = get_job(L, (int64_t)blockIdx.x, local);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 31, g = lane >> 5;
    const int64_t S0 = local * MFMA_ROWS;  // first output row (32-digit block) of the block

    // block range of t, split evenly between the waves
    int64_t tlo = S0 - J.nA32 + 1;
    if (tlo < 0) tlo = 0;
    int64_t thi = S0 + MFMA_ROWS - 1;
    if (thi > J.nB32 - 1) thi = J.nB32 - 1;
    const int64_t tcount = thi >= tlo ? thi - tlo + 1 : 0;
    const int64_t per = (tcount + MFMA_WAVES - 1) / MFMA_WAVES;
    const int64_t wlo = tlo + wv * per;
    int64_t whi = wlo + per;  // exclusive
    if (whi > thi + 1) whi = thi + 1;
    const int64_t nchunks = (per + MFMA_TC - 1) / MFMA_TC;  // same for every wave

    uint8_t *aw = lds + wv * WBYTES;
    uint8_t *bw = aw + AWIN;

    v16i acc[MFMA_RT];
#pragma unroll
    for (int rt = 0; rt < MFMA_RT; ++rt)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[rt][i] = 0;

    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int64_t tc = wlo + ch * MFMA_TC;
        const int64_t tn = whi - tc < MFMA_TC ? whi - tc : MFMA_TC;  // steps in this chunk (may be <= 0)
        // stage the a window: a indices [32 (S0 - tc - TC + 1), 32 (S0 + ROWS - tc))
        const int64_t abase = J.a_front + 32 * (S0 - tc - MFMA_TC + 1);
        for (int x = lane; x < AWIN / 16; x += 64) {
            uint4 v = make_uint4(0, 0, 0, 0);
            if (tn > 0) v = *reinterpret_cast<const uint4 *>(J.ad + abase + 16 * x);
            *reinterpret_cast<uint4 *>(aw + 16 * x) = v;
        }
        // stage the b window (reversed digits): offsets from LB - 1 - PADB - 32 (tc + TC - 1) - 31
        const int64_t bo_min = J.b_top - 32 * (tc + MFMA_TC - 1) - 31;
        const int64_t bstart = bo_min & ~(int64_t)3;
        for (int x = lane; x < BWIN / 4; x += 64) {
            uint32_t v = 0;
            const int64_t o = bstart + 4 * x;
            if (tn > 0 && o >= 0 && o + 4 <= J.b_len) v = *reinterpret_cast<const uint32_t *>(J.bd + o);
            *reinterpret_cast<uint32_t *>(bw + 4 * x) = v;
        }
        __syncthreads();
        for (int64_t u = 0; u < tn; ++u) {
            const int64_t t = tc + u;
            // B operand: 16 bytes of reversed b at offset b_top - 32 t - m + 16 g (column m)
            const int64_t o = J.b_top - 32 * t - m + 16 * g - bstart;
            const uint32_t *bw32 = reinterpret_cast<const uint32_t *>(bw) + (o >> 2);
            const uint32_t sh = (uint32_t)(o & 3);
            uint32_t w0 = bw32[0], w1 = bw32[1], w2 = bw32[2], w3 = bw32[3], w4 = bw32[4];
            v4i bop;
            bop[0] = (int)__builtin_amdgcn_alignbyte(w1, w0, sh);
            bop[1] = (int)__builtin_amdgcn_alignbyte(w2, w1, sh);
            bop[2] = (int)__builtin_amdgcn_alignbyte(w3, w2, sh);
            bop[3] = (int)__builtin_amdgcn_alignbyte(w4, w3, sh);
#pragma unroll
            for (int rt = 0; rt < MFMA_RT; ++rt) {
                // A operand: a[32 (S0 + 32 rt + m - t) + 16 g .. + 15] (row m of tile rt)
                const int64_t ao = 32 * (32 * rt + m - u + MFMA_TC - 1) + 16 * g;
                const v4i aop = *reinterpret_cast<const v4i *>(aw + ao);
                acc[rt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(aop, bop, acc[rt], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // add the waves' digit sums into limb accumulators: digit k of the block (k = 32 row + col)
    // sits at bit 7 k; its lower 32 bits after the shift go to limb 7k >> 5 (X), the rest to the
    // next limb (Y)
    unsigned long long *X = reinterpret_cast<unsigned long long *>(lds);
    unsigned long long *Y = X + MFMA_LIMBS;
    for (int x = tid; x < 2 * MFMA_LIMBS; x += MFMA_TPB) X[x] = 0ull;
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < MFMA_RT; ++rt) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = 32 * rt + 8 * (i >> 2) + 4 * g + (i & 3);
            const int k = 32 * row + m;
            const uint64_t v = (uint64_t)(uint32_t)acc[rt][i] << ((7 * k) & 31);
            const int j = (7 * k) >> 5;
            if (v) {
                atomicAdd(&X[j], (unsigned long long)(uint32_t)v);
                if (v >> 32) atomicAdd(&Y[j], (unsigned long long)(v >> 32));
            }
        }
    }
    __syncthreads();
    uint32_t *out = J.cols + 3 * (local * MFMA_LIMBS);
    for (int j = tid; j < MFMA_LIMBS; j += MFMA_TPB) {
        const uint64_t xv = X[j], yv = Y[j];
        const uint64_t rest = (xv >> 32) + yv;  // weight 2^32 relative to limb j
        out[3 * j + 0] = (uint32_t)xv;
        out[3 * j + 1] = (uint32_t)rest;
        out[3 * j + 2] = (uint32_t)(rest >> 32);
    }
}

hipError_t launch_digitize(const Launch<DigitJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(digitize_kernel, dim3((unsigned)L.total_blocks), dim3(256), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_mul_mfma(const Launch<MfmaJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(mul_mfma_kernel, dim3((unsigned)L.total_blocks), dim3(MFMA_TPB), 0, s, L);
    return hipGetLastError();
}

}  // namespace ks
