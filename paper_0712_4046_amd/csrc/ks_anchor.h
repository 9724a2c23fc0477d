// ks_anchor.h -- the anchor of a reconstruction segment: the exact coefficient h_{sK-1} (plus
// the slot constant) as a dot product of the inputs, one block per anchor.  Used by the
// anchor kernel and by the fused pack-and-anchor launch (anchors read only the inputs).
#pragma once

#include "ks_device.h"

namespace ks {

template <int W>
__device__ __forceinline__ bool load_mag(const uint32_t *c, bool sgn, uint32_t (&m)[W]) {
    bool neg = sgn && (c[W - 1] >> 31);
    uint64_t carry = 1;
#pragma unroll
    for (int t = 0; t < W; ++t) {
        uint32_t x = c[t];
        if (neg) {
            uint64_t s = (uint64_t)(uint32_t)~x + carry;
            m[t] = (uint32_t)s;
            carry = s >> 32;
        } else {
            m[t] = x;
        }
    }
    return neg;
}

// One block computes one anchor: block `local` of anchor job J.
template <int W>
__device__ __forceinline__ void anchor_block(const AnchorJob &J, int64_t local) {
    constexpr int AW = 2 * W + 2;
    __shared__ uint32_t s_acc[ANCHOR_TPB / 64][AW];
    const int64_t s = local + 1;
    const int64_t k = J.kstep * (s * J.K - 1) + J.par;
    int64_t lo = k - (J.lg - 1);
    if (lo < 0) lo = 0;
    int64_t hi = k < J.lf - 1 ? k : J.lf - 1;
    const bool sgn = J.sgn != 0;

    uint32_t acc[AW];
#pragma unroll
    for (int t = 0; t < AW; ++t) acc[t] = 0;
    // ANCHOR_U terms per round, their loads issued together (clamped addresses, masked terms)
    constexpr int U = 4;
    for (int64_t i0 = lo + threadIdx.x; i0 <= hi; i0 += U * ANCHOR_TPB) {
        uint32_t a[U][W], b[U][W];
        bool na[U], nb[U], live[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t i = i0 + (int64_t)q * ANCHOR_TPB;
            live[q] = i <= hi;
            const int64_t ii = live[q] ? i : lo;
            na[q] = load_mag<W>(J.f + ii * W, sgn, a[q]);
            nb[q] = load_mag<W>(J.g + (k - ii) * W, sgn, b[q]);
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (!live[q]) continue;
            uint32_t p[2 * W];
#pragma unroll
            for (int t = 0; t < 2 * W; ++t) p[t] = 0;
#pragma unroll
            for (int x = 0; x < W; ++x) {
                uint64_t c = 0;
#pragma unroll
                for (int y = 0; y < W; ++y) {
                    uint64_t tt = (uint64_t)a[q][x] * b[q][y] + p[x + y] + c;
                    p[x + y] = (uint32_t)tt;
                    c = tt >> 32;
                }
                p[x + W] = (uint32_t)c;
            }
            if (na[q] != nb[q]) {
                uint64_t br = 0;
#pragma unroll
                for (int t = 0; t < AW; ++t) {
                    uint64_t d = (uint64_t)acc[t] - (t < 2 * W ? p[t] : 0u) - br;
                    acc[t] = (uint32_t)d;
                    br = (d >> 63) & 1u;
                }
            } else {
                uint64_t c = 0;
#pragma unroll
                for (int t = 0; t < AW; ++t) {
                    uint64_t sm = (uint64_t)acc[t] + (t < 2 * W ? p[t] : 0u) + c;
                    acc[t] = (uint32_t)sm;
                    c = sm >> 32;
                }
            }
        }
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
