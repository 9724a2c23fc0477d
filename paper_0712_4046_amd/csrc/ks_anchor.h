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
    // U terms per round, their loads issued together (clamped addresses; a dead term's f is
    // zeroed, which also clears its sign)
    constexpr int U = 4;
    for (int64_t i0 = lo + threadIdx.x; i0 <= hi; i0 += U * ANCHOR_TPB) {
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
#pragma unroll
        for (int q = 0; q < U; ++q) {
#pragma unroll
            for (int x = 0; x < W; ++x) a[q][x] = live[q] ? a[q][x] : 0u;
#pragma unroll
            for (int x = 0; x < W; ++x)
#pragma unroll
                for (int y = 0; y < W; ++y) mac96(clo[x + y], chi[x + y], a[q][x], b[q][y]);
            if (sgn) {
                const bool nf = a[q][W - 1] >> 31, ng = b[q][W - 1] >> 31;
#pragma unroll
                for (int t = 0; t < W; ++t)
                    corr[t] += (uint64_t)(nf ? b[q][t] : 0u) + (ng ? a[q][t] : 0u);
                nn += (nf && ng) ? 1u : 0u;
            }
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

}  // namespace ks
