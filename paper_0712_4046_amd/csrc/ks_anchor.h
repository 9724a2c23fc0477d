// ks_anchor.h -- the anchor of a reconstruction segment: the exact coefficient h_{sK-1} (plus
// the slot constant) as a dot product of the inputs, one block per anchor.  Used by the
// anchor kernel and by the fused pack-and-anchor launch (anchors read only the inputs).
#pragma once

#include "ks_device.h"

namespace ks {

// Raw limbs of a W-limb coefficient.  A signed coefficient is c = C - n 2^(32W), C the limbs
// read unsigned and n its sign bit, so over a dot product
//   sum f_i g_j = sum F_i G_j - 2^(32W) (sum n_i G_j + sum m_j F_i) + 2^(64W) sum n_i m_j,
// every sum of nonnegative terms: the loop needs no per-term negation, and the result is
// exact modulo 2^(32 AW), which holds the anchor.
template <int W>
__device__ __forceinline__ void load_raw(const uint32_t *c, uint32_t (&m)[W]) {
    ldg_words<W>(c, m);
}

// p + off bytes, off unsigned 32-bit
__device__ __forceinline__ const uint32_t *byte_at(const uint32_t *p, uint32_t off) {
    return reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(p) + off);
}

// acc (n words, mod 2^(32 n)) += v 2^(32 off), v given as words v[0..nv)
template <int N, int NV>
__device__ __forceinline__ void add_words(uint32_t (&acc)[N], int off, const uint32_t (&v)[NV]) {
    uint64_t c = 0;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        const int q = t - off;
        const uint32_t x = (q >= 0 && q < NV) ? v[q] : 0u;
        const uint64_t sm = (uint64_t)acc[t] + x + c;
        acc[t] = (uint32_t)sm;
        c = sm >> 32;
    }
}

template <int N, int NV>
__device__ __forceinline__ void sub_words(uint32_t (&acc)[N], int off, const uint32_t (&v)[NV]) {
    uint64_t br = 0;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        const int q = t - off;
        const uint32_t x = (q >= 0 && q < NV) ? v[q] : 0u;
        const uint64_t d = (uint64_t)acc[t] - x - br;
        acc[t] = (uint32_t)d;
        br = (d >> 63) & 1u;
    }
}

// acc (AW words) += 2^(32 c) clo/chi (the NC 96-bit column sums) and the sign corrections
template <int W>
__device__ __forceinline__ void anchor_collect(uint32_t (&acc)[2 * W + 2], const uint64_t (&clo)[2 * W - 1],
                                               const uint32_t (&chi)[2 * W - 1], const uint64_t (&corr)[W],
                                               uint32_t nn, bool sgn) {
    constexpr int AW = 2 * W + 2, NC = 2 * W - 1;
#pragma unroll
    for (int t = 0; t < AW; ++t) acc[t] = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t v[3] = {(uint32_t)clo[c], (uint32_t)(clo[c] >> 32), chi[c]};
        add_words(acc, c, v);
    }
    if (sgn) {
#pragma unroll
        for (int t = 0; t < W; ++t) {
            const uint32_t v[2] = {(uint32_t)corr[t], (uint32_t)(corr[t] >> 32)};
            sub_words(acc, W + t, v);
        }
        const uint32_t v[1] = {nn};
        add_words(acc, 2 * W, v);
    }
}

// one term f_i g_j into a column-sum accumulator (and its sign corrections)
template <int W>
__device__ __forceinline__ void anchor_term(uint64_t (&clo)[2 * W - 1], uint32_t (&chi)[2 * W - 1],
                                            uint64_t (&corr)[W], uint32_t &nn, const uint32_t *a,
                                            const uint32_t *b, bool sgn) {
#pragma unroll
    for (int x = 0; x < W; ++x)
#pragma unroll
        for (int y = 0; y < W; ++y) mac96(clo[x + y], chi[x + y], a[x], b[y]);
    if (sgn) {
        const bool nf = a[W - 1] >> 31, ng = b[W - 1] >> 31;
#pragma unroll
        for (int t = 0; t < W; ++t) corr[t] += (uint64_t)(nf ? b[t] : 0u) + (ng ? a[t] : 0u);
        nn += (nf && ng) ? 1u : 0u;
    }
}

// One block computes one anchor: block `local` of anchor job J.  Each lane keeps a 96-bit sum
// per limb column of the products (mac96), plus the sign corrections above.
template <int W>
__device__ __forceinline__ void anchor_block(const AnchorJob &J, int64_t local) {
    constexpr int AW = 2 * W + 2, NC = 2 * W - 1;
    __shared__ uint32_t s_acc[ANCHOR_TPB / 64][AW];
    const int64_t s = local + 1;
    const int64_t k = J.kstep * (s * J.K - 1) + J.par;
    int64_t lo = k - (J.lg - 1);
    if (lo < 0) lo = 0;
    int64_t hi = k < J.lf - 1 ? k : J.lf - 1;
    const bool sgn = J.sgn != 0;

    uint64_t clo[NC];
    uint32_t chi[NC];
    uint64_t corr[W];
    uint32_t nn = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) { clo[c] = 0; chi[c] = 0; }
#pragma unroll
    for (int t = 0; t < W; ++t) corr[t] = 0;
    // U terms per round, their loads issued together.  Whole rounds (every term inside [lo, hi])
    // need no guards and address f and g by 32-bit word offsets that move by constants; the
    // last, partial round clamps its addresses and zeroes a dead term's f (which also clears
    // its sign).
    constexpr int U = 4;
    constexpr uint32_t STEP = (uint32_t)(ANCHOR_TPB * W * 4);  // bytes between a thread's terms
    int64_t i0 = lo + threadIdx.x;
    if (i0 + (U - 1) * ANCHOR_TPB <= hi) {
        // byte offsets from f and g (below 2^32 for inputs of less than 2^27 coefficients):
        // the loads take a scalar base and a 32-bit vector offset, no 64-bit address arithmetic
        uint32_t fo = (uint32_t)(i0 * W * 4), go = (uint32_t)((k - i0) * W * 4);
        for (; i0 + (U - 1) * ANCHOR_TPB <= hi; i0 += U * ANCHOR_TPB, fo += U * STEP, go -= U * STEP) {
            uint32_t a[U][W], b[U][W];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                load_raw<W>(byte_at(J.f, fo + q * STEP), a[q]);
                load_raw<W>(byte_at(J.g, go - q * STEP), b[q]);
            }
            __builtin_amdgcn_sched_barrier(0);  // all of the round's loads in flight first
#pragma unroll
            for (int q = 0; q < U; ++q) anchor_term<W>(clo, chi, corr, nn, a[q], b[q], sgn);
        }
    }
    if (i0 <= hi) {
        uint32_t a[U][W], b[U][W];
        bool live[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t i = i0 + (int64_t)q * ANCHOR_TPB;
            live[q] = i <= hi;
            const int64_t ii = live[q] ? i : lo;
            load_raw<W>(J.f + ii * W, a[q]);
            load_raw<W>(J.g + (k - ii) * W, b[q]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < U; ++q) {
#pragma unroll
            for (int x = 0; x < W; ++x) a[q][x] = live[q] ? a[q][x] : 0u;
            anchor_term<W>(clo, chi, corr, nn, a[q], b[q], sgn);
        }
    }
    uint32_t acc[AW];
#pragma unroll
    for (int t = 0; t < AW; ++t) acc[t] = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t v[3] = {(uint32_t)clo[c], (uint32_t)(clo[c] >> 32), chi[c]};
        add_words(acc, c, v);
    }
    if (sgn) {
#pragma unroll
        for (int t = 0; t < W; ++t) {
            const uint32_t v[2] = {(uint32_t)corr[t], (uint32_t)(corr[t] >> 32)};
            sub_words(acc, W + t, v);
        }
        const uint32_t v[1] = {nn};
        add_words(acc, 2 * W, v);
    }
    // wave reduction, then across waves
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t o[AW];
#pragma unroll
        for (int t = 0; t < AW; ++t) o[t] = (uint32_t)__shfl_down((int)acc[t], d, 64);
        uint64_t c = 0;
#pragma unroll
        for (int t = 0; t < AW; ++t) {
            uint64_t sm = (uint64_t)acc[t] + o[t] + c;
            acc[t] = (uint32_t)sm;
            c = sm >> 32;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int t = 0; t < AW; ++t) s_acc[wv][t] = acc[t];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < ANCHOR_TPB / 64; ++q) {
            uint64_t c = 0;
#pragma unroll
            for (int t = 0; t < AW; ++t) {
                uint64_t sm = (uint64_t)acc[t] + s_acc[q][t] + c;
                acc[t] = (uint32_t)sm;
                c = sm >> 32;
            }
        }
        if (J.off_bit >= 0) {
            uint64_t c = 0;
#pragma unroll
            for (int t = 0; t < AW; ++t) {
                uint32_t add = ((J.off_bit >> 5) == t) ? (1u << (J.off_bit & 31)) : 0u;
                uint64_t sm = (uint64_t)acc[t] + add + c;
                acc[t] = (uint32_t)sm;
                c = sm >> 32;
            }
        }
        uint32_t *dst = J.anchors + s * J.aw;
#pragma unroll
        for (int t = 0; t < AW; ++t) dst[t] = acc[t];
    }
}

// Two anchors in one pass: h_k for job J's chain (anchor s) and h_{k+1} for its second chain
// (anchor s of anchors2, when s < nseg2).  Both read f_i against neighbouring coefficients of
// g, so the pair costs one stream of the inputs instead of two: the two g coefficients of a
// term, g_{k-i} and g_{k+1-i}, come in one vector load.  Terms where only one of the two g's
// lies inside g (i = k - lg + 1 for h_k, i = k + 1 for h_{k+1}) are added by thread 0.
template <int W>
__device__ __forceinline__ void anchor_pair_block(const AnchorJob &J, int64_t local) {
    constexpr int AW = 2 * W + 2, NC = 2 * W - 1;
    __shared__ uint32_t s_acc2[ANCHOR_TPB / 64][2][AW];
    const int64_t s = local + 1;
    const int64_t k = J.kstep * (s * J.K - 1) + J.par;
    int64_t lo = k - (J.lg - 2);  // g_{k-i} and g_{k+1-i} both inside g
    if (lo < 0) lo = 0;
    const int64_t hi = k < J.lf - 1 ? k : J.lf - 1;
    const bool sgn = J.sgn != 0;
    uint64_t clo[2][NC], corr[2][W];
    uint32_t chi[2][NC], nn[2] = {0u, 0u};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int c = 0; c < NC; ++c) { clo[h][c] = 0; chi[h][c] = 0; }
#pragma unroll
        for (int t = 0; t < W; ++t) corr[h][t] = 0;
    }
    constexpr int U = 4;
    constexpr uint32_t STEP = (uint32_t)(ANCHOR_TPB * W * 4);
    int64_t i0 = lo + threadIdx.x;
    if (i0 + (U - 1) * ANCHOR_TPB <= hi) {  // whole rounds, unguarded (as in anchor_block)
        uint32_t fo = (uint32_t)(i0 * W * 4), go = (uint32_t)((k - i0) * W * 4);
        for (; i0 + (U - 1) * ANCHOR_TPB <= hi; i0 += U * ANCHOR_TPB, fo += U * STEP, go -= U * STEP) {
            uint32_t a[U][W], b[U][2 * W];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                load_raw<W>(byte_at(J.f, fo + q * STEP), a[q]);
                ldg_words<2 * W>(byte_at(J.g, go - q * STEP), b[q]);  // g_{k-i}, g_{k-i+1}
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                anchor_term<W>(clo[0], chi[0], corr[0], nn[0], a[q], b[q], sgn);
                anchor_term<W>(clo[1], chi[1], corr[1], nn[1], a[q], b[q] + W, sgn);
            }
        }
    }
    if (i0 <= hi) {  // the last, partial round
        uint32_t a[U][W], b[U][2 * W];
        bool live[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t i = i0 + (int64_t)q * ANCHOR_TPB;
            live[q] = i <= hi;
            const int64_t ii = live[q] ? i : lo;
            load_raw<W>(J.f + ii * W, a[q]);
            ldg_words<2 * W>(J.g + (k - ii) * W, b[q]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < U; ++q) {
#pragma unroll
            for (int x = 0; x < W; ++x) a[q][x] = live[q] ? a[q][x] : 0u;
            anchor_term<W>(clo[0], chi[0], corr[0], nn[0], a[q], b[q], sgn);
            anchor_term<W>(clo[1], chi[1], corr[1], nn[1], a[q], b[q] + W, sgn);
        }
    }
    if (threadIdx.x == 0) {
        const int64_t ie = k - (J.lg - 1);  // h_k's term with g_{lg-1}
        if (ie >= 0 && ie <= hi) {
            uint32_t a[W], b[W];
            load_raw<W>(J.f + ie * W, a);
            load_raw<W>(J.g + (J.lg - 1) * W, b);
            anchor_term<W>(clo[0], chi[0], corr[0], nn[0], a, b, sgn);
        }
        if (k + 1 <= J.lf - 1 && k + 1 >= 0) {  // h_{k+1}'s term with g_0
            uint32_t a[W], b[W];
            load_raw<W>(J.f + (k + 1) * W, a);
            load_raw<W>(J.g, b);
            anchor_term<W>(clo[1], chi[1], corr[1], nn[1], a, b, sgn);
        }
    }
    uint32_t acc[2][AW];
    anchor_collect<W>(acc[0], clo[0], chi[0], corr[0], nn[0], sgn);
    anchor_collect<W>(acc[1], clo[1], chi[1], corr[1], nn[1], sgn);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t o[AW];
#pragma unroll
            for (int t = 0; t < AW; ++t) o[t] = (uint32_t)__shfl_down((int)acc[h][t], d, 64);
            uint64_t c = 0;
#pragma unroll
            for (int t = 0; t < AW; ++t) {
                const uint64_t sm = (uint64_t)acc[h][t] + o[t] + c;
                acc[h][t] = (uint32_t)sm;
                c = sm >> 32;
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int t = 0; t < AW; ++t) s_acc2[wv][h][t] = acc[h][t];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            for (int q = 1; q < ANCHOR_TPB / 64; ++q) {
                uint64_t c = 0;
#pragma unroll
                for (int t = 0; t < AW; ++t) {
                    const uint64_t sm = (uint64_t)acc[h][t] + s_acc2[q][h][t] + c;
                    acc[h][t] = (uint32_t)sm;
                    c = sm >> 32;
                }
            }
            if (J.off_bit >= 0) {
                uint64_t c = 0;
#pragma unroll
                for (int t = 0; t < AW; ++t) {
                    const uint32_t add = ((J.off_bit >> 5) == t) ? (1u << (J.off_bit & 31)) : 0u;
                    const uint64_t sm = (uint64_t)acc[h][t] + add + c;
                    acc[h][t] = (uint32_t)sm;
                    c = sm >> 32;
                }
            }
        }
        uint32_t *dst = J.anchors + s * J.aw;
#pragma unroll
        for (int t = 0; t < AW; ++t) dst[t] = acc[0][t];
        if (s < J.nseg2) {
            uint32_t *dst2 = J.anchors2 + s * J.aw;
#pragma unroll
            for (int t = 0; t < AW; ++t) dst2[t] = acc[1][t];
        }
    }
}

}  // namespace ks
