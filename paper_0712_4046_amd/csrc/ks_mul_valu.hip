// ks_mul_valu.hip -- integer products on the vector ALU (the multiplications of paper
// Sections 3.1-3.4, i.e. M(b) for KS1 and the two or four smaller products of the multipoint
// variants).
//
// Product scanning: output limb column k of A*B is sum_i a_i b_{k-i}.  A block owns MUL_T
// consecutive columns (MUL_R adjacent columns per lane) and its MUL_WAVES waves split the
// i range between them in interleaved chunks of MUL_CI, so even one product of a few
// thousand limbs fills the GPU without partial sums leaving the block.  Each lane keeps a
// 96-bit sum per column: v_mad_u64_u32 accumulates the 32x32-bit product into 64 bits and
// hands its carry to a v_addc into the top 32 bits.  Operand chunks go through LDS; a_i is
// read as a broadcast, b as one aligned 64-bit read per MUL_R steps (a lane's columns see a
// sliding window of b).
//
// Output: per column the 96-bit sum as three 32-bit pieces (weights 2^0, 2^32, 2^64); the
// consumer (normalize_kernel) adds piece p of column k into limb k + p.
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

// MUL_R consecutive LDS words (16-byte aligned for 4, 8-byte aligned for 2) in one read
__device__ __forceinline__ void lds_words(const uint32_t *p, uint32_t (&v)[MUL_R]) {
    static_assert(MUL_R == 2 || MUL_R == 4, "LDS reads of 2 or 4 words");
    if constexpr (MUL_R == 4) {
        const uint4 x = *reinterpret_cast<const uint4 *>(p);
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    } else {
        const uint2 x = *reinterpret_cast<const uint2 *>(p);
        v[0] = x.x;
        v[1] = x.y;
    }
}

// WAVE = false: a block owns one MUL_T-column tile and its waves split the i range (large
// products).  WAVE = true: every wave owns one tile and runs its whole i range alone, and the
// waves of a block take consecutive tiles of the launch, of one product or of several (small
// products, whose short i ranges would leave most of a block's waves idle); a job's blocks
// then count tiles, not thread blocks.
template <bool WAVE>
__global__ __launch_bounds__(MUL_TPB) void mul_valu_kernel(Launch<MulJob> L) {
    __shared__ __attribute__((aligned(16))) uint32_t sa[MUL_WAVES][MUL_CI];
    __shared__ __attribute__((aligned(16))) uint32_t sb[MUL_WAVES][MUL_T + MUL_CI];
    __shared__ uint64_t s_lo[WAVE ? 1 : MUL_WAVES][MUL_T];
    __shared__ uint32_t s_hi[WAVE ? 1 : MUL_WAVES][MUL_T];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t item = WAVE ? (int64_t)blockIdx.x * MUL_WAVES + wv : (int64_t)blockIdx.x;
    if (WAVE && item >= L.total_blocks) return;  // no block-wide barrier in this mode
    int64_t local;
    const MulJob J = get_job(L, item, local);
    const int64_t k0 = local * MUL_T;
    int64_t ilo = k0 - J.nb + 1;
    if (ilo < 0) ilo = 0;
    int64_t ihi = J.na < k0 + MUL_T ? J.na : k0 + MUL_T;

    uint64_t lo[MUL_R];
    uint32_t hi[MUL_R];
#pragma unroll
    for (int r = 0; r < MUL_R; ++r) { lo[r] = 0; hi[r] = 0; }

    // block mode: the waves take interleaved chunks of the i range (wave w runs chunks w,
    // w + WAVES, ...); wave mode: the wave runs every chunk.  The next chunk's operands are
    // loaded into registers while the current one is computed.
    const int64_t span = WAVE ? (int64_t)MUL_CI : (int64_t)MUL_WAVES * MUL_CI;
    const int64_t first = WAVE ? 0 : (int64_t)wv * MUL_CI;
    const int64_t niter = ihi > ilo ? (ihi - ilo + span - 1) / span : 0;
    const int base = lane * MUL_R + MUL_CI - MUL_R;
    constexpr int NA = MUL_CI / 64, NB = (MUL_T + MUL_CI) / 64;
    static_assert(MUL_CI % 64 == 0 && (MUL_T + MUL_CI) % 64 == 0, "staging is 64 words per lane round");
    uint32_t ra[NA], rb[NB];
    auto fetch = [&](int64_t it) {
        const int64_t c0 = ilo + it * span + first;
        const bool active = c0 < ihi;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int64_t i = c0 + lane + 64 * q;
            ra[q] = (active && i < ihi) ? ldg(J.a + i) : 0u;
        }
        const int64_t bfirst = k0 - c0 - MUL_CI + 1;  // b index held in sb[wv][0]
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int64_t bi = bfirst + lane + 64 * q;
            rb[q] = (active && bi >= 0 && bi < J.nb) ? ldg(J.b + bi) : 0u;
        }
    };
    // the staging area of a wave is its own: in wave mode the wave's LDS accesses, performed
    // in issue order, need only a compiler barrier between writing and reading
    auto sync = [&]() {
        if (WAVE) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else {
            __syncthreads();
        }
    };
    if (niter > 0) fetch(0);
    for (int64_t it = 0; it < niter; ++it) {
        const int64_t c0 = ilo + it * span + first;
        const bool active = c0 < ihi;
#pragma unroll
        for (int q = 0; q < NA; ++q) sa[wv][lane + 64 * q] = ra[q];
#pragma unroll
        for (int q = 0; q < NB; ++q) sb[wv][lane + 64 * q] = rb[q];
        sync();
        if (it + 1 < niter) fetch(it + 1);
        if (active) {
            // E[idx] = sb[base - x0 + idx]; column r at step x0 + u uses E[R - 1 + r - u].  The
            // chunk's steps at or beyond ihi read a_i = 0 (staged as zeros): the loop stops at the
            // last step that meets a (the tail chunk of a short i range is often a few steps)
            constexpr int XG = 4 * MUL_R;  // steps per unrolled group (MUL_CI is a multiple)
            static_assert(MUL_CI % XG == 0, "whole groups of steps per chunk");
            const int xlen = (int)(ihi - c0 < (int64_t)MUL_CI ? ihi - c0 : (int64_t)MUL_CI);
            const int xend = (xlen + XG - 1) / XG * XG;
            uint32_t ehi[MUL_R];
            lds_words(&sb[wv][base + MUL_R], ehi);
            for (int xg = 0; xg < xend; xg += XG) {
#pragma unroll
                for (int xu = 0; xu < XG; xu += MUL_R) {
                    const int x0 = xg + xu;
                    uint32_t elo[MUL_R], A[MUL_R], E[2 * MUL_R];
                    lds_words(&sb[wv][base - x0], elo);
                    lds_words(&sa[wv][x0], A);
#pragma unroll
                    for (int t = 0; t < MUL_R; ++t) {
                        E[t] = elo[t];
                        E[MUL_R + t] = ehi[t];
                    }
#pragma unroll
                    for (int u = 0; u < MUL_R; ++u)
#pragma unroll
                        for (int r = 0; r < MUL_R; ++r) mac96(lo[r], hi[r], A[u], E[MUL_R - 1 + r - u]);
#pragma unroll
                    for (int t = 0; t < MUL_R; ++t) ehi[t] = elo[t];
                }
            }
        }
        sync();
    }

    if (WAVE) {
        // the wave's own sums, three 32-bit pieces per column
#pragma unroll
        for (int r = 0; r < MUL_R; ++r) {
            uint32_t *o = J.cols + 3 * (k0 + lane * MUL_R + r);
            o[0] = (uint32_t)lo[r];
            o[1] = (uint32_t)(lo[r] >> 32);
            o[2] = hi[r];
        }
        return;
    }
    // add the waves' 96-bit sums and store them as three 32-bit pieces per column
#pragma unroll
    for (int r = 0; r < MUL_R; ++r) {
        s_lo[WAVE ? 0 : wv][lane * MUL_R + r] = lo[r];
        s_hi[WAVE ? 0 : wv][lane * MUL_R + r] = hi[r];
    }
    __syncthreads();
    for (int t = tid; t < MUL_T; t += MUL_TPB) {
        uint64_t l = 0;
        uint32_t h = 0;
#pragma unroll
        for (int w = 0; w < (WAVE ? 1 : MUL_WAVES); ++w) {
            const uint64_t x = s_lo[w][t];
            l += x;
            h += (l < x ? 1u : 0u) + s_hi[w][t];
        }
        uint32_t *o = J.cols + 3 * (k0 + t);
        o[0] = (uint32_t)l;
        o[1] = (uint32_t)(l >> 32);
        o[2] = h;
    }
}

hipError_t launch_mul_valu(const Launch<MulJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    ks_launch(mul_valu_kernel<false>, dim3((unsigned)L.total_blocks), dim3(MUL_TPB), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_mul_valu_wave(const Launch<MulJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    const int64_t blocks = (L.total_blocks + MUL_WAVES - 1) / MUL_WAVES;
    ks_launch(mul_valu_kernel<true>, dim3((unsigned)blocks), dim3(MUL_TPB), 0, s, L);
    return hipGetLastError();
}

}  // namespace ks
