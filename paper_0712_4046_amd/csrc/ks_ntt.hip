// ks_ntt.hip -- integer products through number-theoretic transforms, for long operands.
//
// The paper's cost model (Section 1) sets M(b) against 4 M(b/4); for very long operands the
// integer product itself should be quasi-linear, which is what this engine provides.  An
// operand of n limbs (its unsigned reading; the recombination corrects two's-complement signs)
// is cut into np = ceil(32 n / w) pieces of w bits, and the pieces of a and b are convolved:
// c_m = sum_i a'_i b'_{m-i}, so that A B = sum_m c_m 2^(w m).  The convolution is computed
// modulo P0 = 119 2^23 + 1 and P1 = 107 2^23 + 1 by transforms of length N = 2^k >= npa + npb - 1
// and joined by the Chinese remainder theorem; the planner picks w so that every c_m stays
// below P0 P1 > 2^59 (2w + log2 min(npa, npb) <= 59), which makes the joined value exact.
//
// A product's transforms of length N = N1 N2 run in three steps (each one launch over every
// job) and a join:
//   forward columns  per operand, N2 transforms of length N1 over the stride-N2 columns
//                    x[N2 n1 + n2], then the twiddle w_N^(n2 k1) (for the second operand times
//                    R^2 / N, the inverse's scale); stored row-wise (row k1, N2 columns)
//   rows             per product, N1 transforms of length N2 over the rows of both operands,
//                    their pointwise product (Montgomery), the inverse row transforms and the
//                    inverse twiddle
//   inverse columns  the inverse column transforms, the residues of the convolution terms
//                    written in order (in place)
//   join             the two residues of each term joined by the Chinese remainder theorem,
//                    the terms gathered into 96-bit limb columns for the recombination
// Forward transforms are decimation in frequency (natural order in, bit-reversed out) and the
// inverse ones decimation in time (bit-reversed in, natural out), so no step reorders data:
// rows are kept at their bit-reversed positions and the pointwise product pairs equal positions.
// A column block transforms NTT_BLOCK elements in LDS (C = NTT_BLOCK / N1 adjacent columns), a
// row block NTT_BLOCK / 2 elements of each operand (R = NTT_BLOCK / 2 / N2 rows), both in a
// padded layout (a spare word after every 32 elements) with per-stage twiddle tables: radix-4
// passes down to half-size 16, then the last four stages in registers on runs of 16 elements.
//
// Arithmetic: residues of P < 2^30 in 32-bit words; products by Montgomery reduction with
// R = 2^32 (a b R^-1 mod P), twiddles kept in Montgomery form so that multiplying a residue by
// one returns the plain product.  Residues stay partly reduced between butterflies (after
// D. Harvey, "Faster arithmetic for number-theoretic transforms", 2014): the forward
// butterflies take and give values below 2P, the inverse ones below 4P, and a product is
// left below 2P (no final subtraction), so a butterfly costs three multiply-adds and five
// additions, subtractions or minima.  Powers of a root of unity of order 2^23 come from two
// tables of 4096 entries per prime (w^e = w^(4096 hi) w^(lo)), and the stage twiddles of the
// transforms in LDS from a table of 4096 per prime and direction, all built on the host once
// per device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "../../include/ks.h"
#include "ks_device.h"
#include "ks_launch.h"
#include "ks_plan.h"

namespace ks {

constexpr int NTT_TAB_LOG = (NTT_ROOT_LOG + 1) / 2;
constexpr int NTT_TAB = 1 << NTT_TAB_LOG;  // 4096 entries per half table
static_assert(2 * NTT_TAB_LOG >= NTT_ROOT_LOG, "two half tables cover the root's powers");
static_assert(NTT_MAX_LOG <= NTT_ROOT_LOG, "the root's order covers the longest transform");
static_assert(4ull * NTT_P0 < (1ull << 32) && 4ull * NTT_P1 < (1ull << 32), "4P fits in a word");
static_assert(NTT_P0 < 2ull * NTT_P1 && (double)NTT_P0 * NTT_P1 > (double)(1ull << 59), "the join's bounds");

// [prime][0: w^(4096 i) R, 1: w^i R][i] mod P (fully reduced)
__device__ uint32_t ntt_tab[2][2][NTT_TAB];
// stage twiddles for transforms of up to 2^12 in LDS: [prime][0: forward, 1: inverse][h + j] =
// w_(2h)^(+-j) R mod P for the stage of half-size h = 2^s (j < h; entry 0 unused).  The entries of
// a half-size do not depend on the transform length, so one table serves every length.
constexpr int NTT_STAGE_TW = 1 << 12;
__device__ uint32_t ntt_stage_tab[2][2][NTT_STAGE_TW];

// w^e R for e in [0, 2^23), w the table root of prime q (fully reduced)
__device__ __forceinline__ uint32_t root_pow(int q, uint32_t e, NttPrime P) {
    return mmul(ntt_tab[q][0][e >> NTT_TAB_LOG], ntt_tab[q][1][e & (NTT_TAB - 1)], P);
}

// The two butterflies on partly reduced residues (P < 2^30).
static_assert(NTT_P0 < (1u << 30) && NTT_P1 < (1u << 30), "partly reduced residues need 4P < 2^32");
// Forward, decimation in frequency: u, v < 2P -> u + v and (u - v) w, both below 2P.
__device__ __forceinline__ void bfly_dif(uint32_t &u, uint32_t &v, uint32_t w, NttPrime P) {
    const uint32_t s = red2(u + v, P.p), d = mmul_lazy(u + 2u * P.p - v, w, P);
    u = s;
    v = d;
}
// Inverse, decimation in time: u, v < 4P -> u + v w and u - v w, both below 4P.
__device__ __forceinline__ void bfly_dit(uint32_t &u, uint32_t &v, uint32_t w, NttPrime P) {
    const uint32_t a = red2(u, P.p), t = mmul_lazy(v, w, P);
    u = a + t;
    v = a + 2u * P.p - t;
}

// ---- the row step's LDS layout --------------------------------------------------------------------
// Element a of a row block lives at word a + (a >> 5): a spare word after every 32.  Then the
// passes are free of bank conflicts (32 lanes of a wave access 32 banks at once): contiguous
// runs of 32 elements keep their banks, and 32 lanes reading runs of 16 elements each (lane l at
// 16 l + i) spread over all 32 banks instead of two.  The twiddles are kept per stage,
// tws[h + j] = w_(2h)^(+-j) R for the stage of half-size h (j < h; tws[0] unused), so that the
// lanes of a pass read consecutive words of them instead of a stride (copied from ntt_stage_tab).
__device__ __forceinline__ int pad_ix(int a) { return a + (a >> 5); }
constexpr int pad_len(int n) { return n + n / 32; }

// one radix-4 pass (stages of half-sizes 2 Hb and Hb, Hb = 2^BL >= 16) in the padded layout:
// the group's elements j + m Hb sit at fixed offsets from element j (its block of 4 Hb
// elements starts at a multiple of 64, so the spare words between them are known).  HALF
// (forward, first pass of a sequence whose upper half is zero): u2 = u3 = 0 are not read, and
// the first stage's butterflies reduce to u2 = u0 w, u3 = u1 w (u0 and u1 stay below 2P).
// NB = 2: the same pass over a second buffer of the same shape, in the same loop (shared
// twiddle reads, twice the independent work between barriers)
template <int LG, int BL, bool INV, int NE, int GAP, bool HALF = false, int NB = 1>
__device__ __forceinline__ void pad_radix4(uint32_t *buf, uint32_t *buf2, const uint32_t *tws, NttPrime P) {
    static_assert(!(HALF && INV), "the zero upper half is a forward-transform input");
    constexpr int hb = 1 << BL, NQ = NE / 4 / NTT_TPB, SS = pad_len(1 << LG) + GAP;
    static_assert(BL >= 4 && BL + 2 <= LG, "radix-4 pass of half-sizes 16 and up");
    constexpr int o1 = hb >= 32 ? hb + hb / 32 : 16, o2 = hb >= 32 ? 2 * o1 : 33, o3 = hb >= 32 ? 3 * o1 : 49;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int g = threadIdx.x + i * NTT_TPB;
        const int seq = g >> (LG - 2), r = g & ((1 << (LG - 2)) - 1);
        const int j = r & (hb - 1);
        const int off = seq * SS + pad_ix(((r >> BL) << (BL + 2)) + j);
        const uint32_t wa0 = tws[2 * hb + j], wa1 = tws[3 * hb + j], wb = tws[hb + j];
        auto one = [&](uint32_t *x) {
        uint32_t u0 = x[0], u1 = x[o1], u2 = HALF ? 0u : x[o2], u3 = HALF ? 0u : x[o3];
        if (HALF) {
            u2 = mmul_lazy(u0, wa0, P);
            u3 = mmul_lazy(u1, wa1, P);
            bfly_dif(u0, u1, wb, P);
            bfly_dif(u2, u3, wb, P);
        } else if (!INV) {
            bfly_dif(u0, u2, wa0, P);
            bfly_dif(u1, u3, wa1, P);
            bfly_dif(u0, u1, wb, P);
            bfly_dif(u2, u3, wb, P);
        } else {
            bfly_dit(u0, u1, wb, P);
            bfly_dit(u2, u3, wb, P);
            bfly_dit(u0, u2, wa0, P);
            bfly_dit(u1, u3, wa1, P);
        }
        x[0] = u0;
        x[o1] = u1;
        x[o2] = u2;
        x[o3] = u3;
        };
        one(buf + off);
        if constexpr (NB == 2) one(buf2 + off);
    }
    __syncthreads();
}

// Transforms of length M = 2^LG over NE elements in the padded layout: NE / M sequences, each
// padded on its own, sequence s at word s (pad_len(M) + GAP) (GAP = 0: one contiguous padded
// array; GAP = 1: columns an odd number of words apart, so that 32 lanes writing one element
// of 32 columns each hit 32 banks).  Forward by decimation in frequency (natural in, bit-reversed
// out, values below 2P), inverse by decimation in time (bit-reversed in, natural out, below 4P):
// a radix-2 stage of half-size M / 2 when LG is odd, radix-4 passes (two stages per LDS round
// trip) down to half-size 16, and the four stages of half-sizes 8, 4, 2, 1 in registers, each
// thread on runs of 16 consecutive elements (their twiddles, w_16^j and its powers, are the same
// for every run).  Forward in that order, the inverse in reverse.  Ends with a barrier.
// HALF (forward only): the upper half of every sequence is zero and is not read, only
// written, by the first stage (the caller need not store those zeros).  NB = 2: two buffers of
// the same shape (buf and buf2) transformed together, pass by pass.
template <int LG, bool INV, int NE, int GAP, bool HALF = false, int NB = 1, bool OUTER = true>
__device__ __forceinline__ void lds_transform_pad(uint32_t *buf, const uint32_t *tws, NttPrime P,
                                                  uint32_t *buf2 = nullptr) {
    constexpr int SS = pad_len(1 << LG) + GAP;
    constexpr bool ODD = ((LG - 4) & 1) != 0;
    constexpr int TOP = LG - 2 - (ODD ? 1 : 0);  // the first (forward) radix-4 pass's BL, even
    static_assert(LG >= 6 && NE % (16 * NTT_TPB) == 0 && NE % (1 << LG) == 0, "padded transform shape");
    auto radix2 = [&]() {  // half-size h = M / 2 >= 32: elements j and j + h, h + h / 32 words apart
        constexpr int h = 1 << (LG - 1), NH = NE / 2 / NTT_TPB, oh = h + h / 32;
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int b = threadIdx.x + i * NTT_TPB;
            const int j = b & (h - 1);
            const int off = (b >> (LG - 1)) * SS + pad_ix(j);
            const uint32_t w = tws[h + j];
            auto one = [&](uint32_t *x) {
                if constexpr (HALF && !INV) {  // v = 0: u stays, v = u w
                    x[oh] = mmul_lazy(x[0], w, P);
                    return;
                }
                uint32_t u = x[0], v = x[oh];
                if (!INV)
                    bfly_dif(u, v, w, P);
                else
                    bfly_dit(u, v, w, P);
                x[0] = u;
                x[oh] = v;
            };
            one(buf + off);
            if constexpr (NB == 2) one(buf2 + off);
        }
        __syncthreads();
    };
    auto tail = [&]() {
        uint32_t t16[8], t8[4], t4[2];
#pragma unroll
        for (int j = 0; j < 8; ++j) t16[j] = tws[8 + j];
#pragma unroll
        for (int j = 0; j < 4; ++j) t8[j] = tws[4 + j];
        t4[0] = tws[2];
        t4[1] = tws[3];
        const uint32_t t2 = tws[1];
#pragma unroll
        for (int i = 0; i < NE / 16 / NTT_TPB; ++i) {
            const int run = threadIdx.x + i * NTT_TPB;  // a run never crosses a spare word
            const int off = (run >> (LG - 4)) * SS + pad_ix((run & ((1 << (LG - 4)) - 1)) << 4);
            auto one = [&](uint32_t *x) {
            uint32_t v[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = x[e];
            if (!INV) {
#pragma unroll
                for (int j = 0; j < 8; ++j) bfly_dif(v[j], v[j + 8], t16[j], P);
#pragma unroll
                for (int b = 0; b < 16; b += 8)
#pragma unroll
                    for (int j = 0; j < 4; ++j) bfly_dif(v[b + j], v[b + j + 4], t8[j], P);
#pragma unroll
                for (int b = 0; b < 16; b += 4)
#pragma unroll
                    for (int j = 0; j < 2; ++j) bfly_dif(v[b + j], v[b + j + 2], t4[j], P);
#pragma unroll
                for (int b = 0; b < 16; b += 2) bfly_dif(v[b], v[b + 1], t2, P);
            } else {
#pragma unroll
                for (int b = 0; b < 16; b += 2) bfly_dit(v[b], v[b + 1], t2, P);
#pragma unroll
                for (int b = 0; b < 16; b += 4)
#pragma unroll
                    for (int j = 0; j < 2; ++j) bfly_dit(v[b + j], v[b + j + 2], t4[j], P);
#pragma unroll
                for (int b = 0; b < 16; b += 8)
#pragma unroll
                    for (int j = 0; j < 4; ++j) bfly_dit(v[b + j], v[b + j + 4], t8[j], P);
#pragma unroll
                for (int j = 0; j < 8; ++j) bfly_dit(v[j], v[j + 8], t16[j], P);
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = v[e];
            };
            one(buf + off);
            if constexpr (NB == 2) one(buf2 + off);
        }
        __syncthreads();
    };
    // !OUTER: the outermost pass (the forward's first, the inverse's last: the radix-2 stage,
    // else the radix-4 pass of half-size 2^TOP) is left to the caller, who holds its elements
    // in registers
    static_assert(OUTER || !HALF, "the zero half enters the outermost pass");
    constexpr bool R2 = ODD && OUTER;
    constexpr int T4 = ODD || OUTER ? TOP : TOP - 2;  // the largest radix-4 pass run here
    if (!INV) {
        constexpr bool H1 = HALF && !ODD;  // the zero half goes into the first radix-4 pass
        if constexpr (R2) radix2();
        if constexpr (T4 >= 10) pad_radix4<LG, 10, false, NE, GAP, H1 && T4 == 10, NB>(buf, buf2, tws, P);
        if constexpr (T4 >= 8) pad_radix4<LG, 8, false, NE, GAP, H1 && T4 == 8, NB>(buf, buf2, tws, P);
        if constexpr (T4 >= 6) pad_radix4<LG, 6, false, NE, GAP, H1 && T4 == 6, NB>(buf, buf2, tws, P);
        if constexpr (T4 >= 4) pad_radix4<LG, 4, false, NE, GAP, H1 && T4 == 4, NB>(buf, buf2, tws, P);
        tail();
    } else {
        tail();
        if constexpr (T4 >= 4) pad_radix4<LG, 4, true, NE, GAP, false, NB>(buf, buf2, tws, P);
        if constexpr (T4 >= 6) pad_radix4<LG, 6, true, NE, GAP, false, NB>(buf, buf2, tws, P);
        if constexpr (T4 >= 8) pad_radix4<LG, 8, true, NE, GAP, false, NB>(buf, buf2, tws, P);
        if constexpr (T4 >= 10) pad_radix4<LG, 10, true, NE, GAP, false, NB>(buf, buf2, tws, P);
        if constexpr (R2) radix2();
    }
}

template <bool INV, int NE, int GAP, bool HALF = false, int NB = 1, bool OUTER = true>
__device__ __forceinline__ void lds_transform_pad_any(int lg, uint32_t *buf, const uint32_t *tws, NttPrime P,
                                                      uint32_t *buf2 = nullptr) {
    switch (lg) {
        case 6: if constexpr (OUTER) lds_transform_pad<6, INV, NE, GAP, HALF, NB>(buf, tws, P, buf2); break;
        case 7: if constexpr (OUTER) lds_transform_pad<7, INV, NE, GAP, HALF, NB>(buf, tws, P, buf2); break;
        case 8: if constexpr (OUTER) lds_transform_pad<8, INV, NE, GAP, HALF, NB>(buf, tws, P, buf2); break;
        case 9: lds_transform_pad<9, INV, NE, GAP, HALF, NB, OUTER>(buf, tws, P, buf2); break;
        case 10: lds_transform_pad<10, INV, NE, GAP, HALF, NB, OUTER>(buf, tws, P, buf2); break;
        case 11: lds_transform_pad<11, INV, NE, GAP, HALF, NB, OUTER>(buf, tws, P, buf2); break;
        default:  // rows only (columns have at most 2^11)
            if constexpr (GAP == 0) lds_transform_pad<12, INV, NE, GAP, HALF, NB, OUTER>(buf, tws, P, buf2);
            break;
    }
}

// piece m of a: bits [w m, w m + w) of its limbs (zero at or above np pieces or n limbs)
__device__ __forceinline__ uint32_t piece_of(uint32_t lo, uint32_t hi, int sh, int w) {
    return (uint32_t)(((((uint64_t)hi << 32) | lo) >> sh) & ((1ull << w) - 1ull));
}

__device__ __forceinline__ uint32_t bitrev(uint32_t r, int bits) { return __builtin_bitreverse32(r) >> (32 - bits); }

// Every thread owns elements tid + NTT_TPB i (i < EPT) of the block; their global loads are
// issued CH at a time before any is used (a rolled loop waits for each load in turn).
constexpr int EPT = NTT_BLOCK / NTT_TPB;
constexpr int CH = 16;

// ---- the four steps ---------------------------------------------------------------------------

// A column block's C columns of N1 residues in LDS: column c at word c SC, SC = pad_len(N1) + 1
// (each column in the padded layout, columns an odd number of words apart), at most
// NTT_COL_BUF words for N1 >= 64.  With 1024 stage twiddles (columns of up to 2^10) a block
// takes 38 KB and four fit on a CU.
constexpr int NTT_COL_BUF = NTT_BLOCK + NTT_BLOCK / 32 + NTT_BLOCK / 64;
static_assert(NTT_MIN_LOG / 2 >= 6, "columns of at least 64");
constexpr int NTT_COLS_TWS_SMALL = 1 << 10, NTT_COLS_TWS = 1 << (NTT_MAX_LOG / 2);

// Column blocks read C words of each row: with C = 16 that is half of a 128-byte line, whose
// other half the next block reads -- both run on one XCD at about the same time (xcd_block), so
// the line comes from HBM once.
template <int Q, int TWS>
__device__ __forceinline__ void fwd_cols_body(const NttJob &J, int64_t local, uint32_t *buf, uint32_t *tws) {
    const int k1 = J.k1, k2 = J.k2, k = k1 + k2;
    const int lc = 13 - k1, C = 1 << lc, SC = pad_len(1 << k1) + 1;  // columns, LDS stride of a column
    const int gl = k - 13;  // log2 of the blocks of one prime (a power of two: no division)
    constexpr int q = Q;
    const int64_t c0 = (local & (((int64_t)1 << gl) - 1)) * C;
    constexpr NttPrime P = ntt_prime_c(Q);
    const int t = threadIdx.x;
    constexpr int TPT = TWS / NTT_TPB;
    uint32_t twf[TPT];  // the stage twiddles, loaded with the pieces
#pragma unroll
    for (int m = 0; m < TPT; ++m) twf[m] = ldg(&ntt_stage_tab[q][0][t + m * NTT_TPB]);
    // element e = t + 256 i of the block: column c = t mod C (256 is a multiple of C), row
    // n1 = t / C + i 256 / C; its piece m = n1 N2 + c0 + c < N <= 2^23 and first bit w m < 2^28
    // fit in 32 bits.  The two words holding the piece come in one 8-byte load (dword alignment
    // is enough) from a word clamped to n - 2, so that every load stays inside the operand and
    // none waits on a branch; the words past the operand (or past np pieces) read as zero.
    const uint32_t w = (uint32_t)J.w, np = (uint32_t)J.np, na = (uint32_t)J.na;
    const uint32_t mt = ((uint32_t)(t >> lc) << k2) + (uint32_t)c0 + (uint32_t)(t & (C - 1));
    const uint32_t mstep = (uint32_t)(NTT_TPB >> lc) << k2;
    const uint32_t last = na >= 2 ? na - 2 : 0;
    uint32_t *bt = buf + (t & (C - 1)) * SC;
    const int n1t = t >> lc, n1s = NTT_TPB >> lc;
    // The pieces at or beyond np are the transform's zero padding (about half of them).  Lane 0
    // of a wave holds its smallest piece index and element i adds i mstep to every lane's, so
    // the chunks of elements from iz on are zero on the whole wave: stored as zeros, unloaded.
    const uint32_t mt0 = __builtin_amdgcn_readfirstlane(mt);
    const int lms = 8 - lc + k2;  // mstep = 2^lms
    const int iz = mt0 >= np ? 0 : (int)min((uint32_t)EPT, (np - mt0 + mstep - 1u) >> lms);
    // When np <= N / 2 every column's upper half (rows n1 >= N1 / 2, this thread's elements
    // i >= EPT / 2, all at or beyond iz) is zero padding: the transform's first stage then
    // writes it without reading it, so it is not stored here.
    const bool half = (uint64_t)np * 2u <= ((uint64_t)1 << k);
    static_assert((EPT / 2) % CH == 0, "the upper half is whole chunks");
    auto load = [&](auto wide) {  // wide: 8-byte loads (an operand of two limbs or more)
#pragma unroll 1
        for (int i0 = 0; i0 < EPT; i0 += CH) {
            if (i0 >= iz) {  // wave-uniform
                if (!half || i0 < EPT / 2) {
#pragma unroll
                    for (int i = 0; i < CH; ++i) bt[pad_ix(n1t + (i0 + i) * n1s)] = 0u;
                }
                continue;
            }
            u32x2 v[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const uint32_t m = mt + (uint32_t)(i0 + i) * mstep, w0 = (w * m) >> 5;
                const uint32_t *src = J.a + min(w0, last);
                if constexpr (decltype(wide)::value)
                    v[i] = *(const __attribute__((address_space(1))) u32x2 *)src;
                else
                    v[i] = u32x2{ldg(src), 0u};
            }
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const uint32_t m = mt + (uint32_t)(i0 + i) * mstep, bit = w * m, w0 = bit >> 5;
                const bool in = m < np;
                const uint32_t lo = in && w0 < na ? (w0 <= last ? v[i].x : v[i].y) : 0u;
                const uint32_t hi = in && w0 + 1 < na ? v[i].y : 0u;
                bt[pad_ix(n1t + (i0 + i) * n1s)] = piece_of(lo, hi, (int)(bit & 31u), (int)w);
            }
        }
    };
    if (na >= 2)
        load(std::true_type{});
    else
        load(std::false_type{});
#pragma unroll
    for (int m = 0; m < TPT; ++m) tws[t + m * NTT_TPB] = twf[m];
    __syncthreads();
    if (half)
        lds_transform_pad_any<false, NTT_BLOCK, 1, true>(k1, buf, tws, P);
    else
        lds_transform_pad_any<false, NTT_BLOCK, 1>(k1, buf, tws, P);
    // twiddle w_N^(n2 k1) and store: each thread takes runs of `cols` adjacent columns of one row
    // (32 elements in all), so the twiddles of a run follow by one multiplication each from its
    // first (w^((c0 + c) kk) = w^((c0 + c_first) kk) (w^kk)^(c - c_first)) and the run is
    // stored with 16-byte stores; LDS reads of adjacent threads fall on adjacent rows
    uint32_t *x = J.x + ((int64_t)q << k);
    const int lcols = lc < 5 ? lc : 5;              // log2 of the run length (columns)
    const int cols = 1 << lcols;
    const int lrpr = lc - lcols;                    // log2 of the threads sharing a row
    const int rows_per_thread = EPT >> lcols;     // runs per thread
    const int sh = NTT_ROOT_LOG - k;
#pragma unroll 1
    for (int rr = 0; rr < rows_per_thread; ++rr) {
        const int run = rr * NTT_TPB + t;           // adjacent threads, adjacent runs (rows)
        const int r = run >> lrpr;
        const int cf = (run - (r << lrpr)) << lcols;
        const uint32_t kk = bitrev((uint32_t)r, k1);
        // (times the job's factor: R^2 / N for the second operand, so that the inverse needs
        // no scaling of its own)
        uint32_t w = mmul(root_pow(q, (uint32_t)(((c0 + cf) * (int64_t)kk) << sh) & ((1u << NTT_ROOT_LOG) - 1u), P),
                          J.kscale[Q], P);
        const uint32_t g = root_pow(q, (uint32_t)(((int64_t)kk) << sh), P);
        uint32_t *dst = x + ((int64_t)r << k2) + c0 + cf;
        const uint32_t *src = buf + cf * SC + pad_ix(r);
        for (int c4 = 0; c4 < cols; c4 += 4) {
            // below 2P.  The running twiddle stays partly reduced, below 2P (w g < 2P^2 < P 2^32
            // with g < P), and so do the products (src w < 4P^2 < P 2^32, as P < 2^30)
            u32x4 v;
            v.x = mmul_lazy(src[c4 * SC], w, P);
            w = mmul_lazy(w, g, P);
            v.y = mmul_lazy(src[(c4 + 1) * SC], w, P);
            w = mmul_lazy(w, g, P);
            v.z = mmul_lazy(src[(c4 + 2) * SC], w, P);
            w = mmul_lazy(w, g, P);
            v.w = mmul_lazy(src[(c4 + 3) * SC], w, P);
            w = mmul_lazy(w, g, P);
            *(__attribute__((address_space(1))) u32x4 *)(dst + c4) = v;
        }
    }
}

template <int TWS>
__global__ __launch_bounds__(NTT_TPB) void ntt_fwd_cols_kernel(Launch<NttJob> L) {
    __shared__ uint32_t buf[NTT_COL_BUF];
    __shared__ uint32_t tws[TWS];
    int64_t local;
    const NttJob J = get_job(L, xcd_block((int64_t)blockIdx.x, L.total_blocks), local);
    if ((local >> (J.k1 + J.k2 - 13)) == 0)  // the prime: a compile-time constant in each body
        fwd_cols_body<0, TWS>(J, local, buf, tws);
    else
        fwd_cols_body<1, TWS>(J, local, buf, tws);
}

// The row step of a product: both operands' rows forward, the pointwise product and the
// inverse row transform, in one pass over HBM.  A block takes
// NTT_ROWS_BLOCK residues (R = NTT_ROWS_BLOCK / N2 whole rows) of each operand for one prime.
constexpr int NTT_ROWS_BLOCK = NTT_BLOCK / 2;
constexpr int EPT_R = NTT_ROWS_BLOCK / NTT_TPB;

// the padded position of element t + NTT_TPB m is tp + PSTEP m (NTT_TPB is a multiple of 32)
constexpr int PSTEP = NTT_TPB + NTT_TPB / 32;

// The outermost pass of rows of 2^K2 residues (K2 >= 9) on a thread's own elements: element i
// of the thread sits at t + 256 i of the row block, so its elements of one row are j + 256 a
// (a < GS = 2^(K2-8), j = t), and the pass's groups (half-sizes of 256 and more) lie inside
// them; tw[m] = tws[t + 256 m] of the pass's direction.  The same butterflies as the radix-2
// stage or the radix-4 pass of lds_transform_pad.
template <int K2, bool INV, int TPT>
__device__ __forceinline__ void row_outer_pass(uint32_t (&u)[EPT_R], const uint32_t (&tw)[TPT], NttPrime P) {
    constexpr int GS = 1 << (K2 - 8);
    static_assert(K2 >= 9 && GS <= TPT && EPT_R % GS == 0, "outer pass in registers");
#pragma unroll
    for (int g0 = 0; g0 < EPT_R; g0 += GS) {
        if constexpr ((K2 & 1) != 0) {  // radix-2 stage of half-size 2^(K2-1)
#pragma unroll
            for (int a = 0; a < GS / 2; ++a) {
                if (!INV)
                    bfly_dif(u[g0 + a], u[g0 + a + GS / 2], tw[GS / 2 + a], P);
                else
                    bfly_dit(u[g0 + a], u[g0 + a + GS / 2], tw[GS / 2 + a], P);
            }
        } else {  // radix-4 pass of half-sizes 2^(K2-1) and 2^(K2-2)
#pragma unroll
            for (int a = 0; a < GS / 4; ++a) {
                uint32_t &u0 = u[g0 + a], &u1 = u[g0 + a + GS / 4], &u2 = u[g0 + a + GS / 2], &u3 = u[g0 + a + 3 * GS / 4];
                const uint32_t wa0 = tw[GS / 2 + a], wa1 = tw[3 * GS / 4 + a], wb = tw[GS / 4 + a];
                if (!INV) {
                    bfly_dif(u0, u2, wa0, P);
                    bfly_dif(u1, u3, wa1, P);
                    bfly_dif(u0, u1, wb, P);
                    bfly_dif(u2, u3, wb, P);
                } else {
                    bfly_dit(u0, u1, wb, P);
                    bfly_dit(u2, u3, wb, P);
                    bfly_dit(u0, u2, wa0, P);
                    bfly_dit(u1, u3, wa1, P);
                }
            }
        }
    }
}

template <bool INV, int TPT>
__device__ __forceinline__ void row_outer(int k2, uint32_t (&u)[EPT_R], const uint32_t (&tw)[TPT], NttPrime P) {
    switch (k2) {
        case 9: row_outer_pass<9, INV>(u, tw, P); break;
        case 10: row_outer_pass<10, INV>(u, tw, P); break;
        case 11: if constexpr (TPT >= 8) row_outer_pass<11, INV>(u, tw, P); break;
        case 12: if constexpr (TPT >= 16) row_outer_pass<12, INV>(u, tw, P); break;
        default: break;
    }
}

template <int Q, int TWS>
__device__ __forceinline__ void rows_body(const NttJob &J, int64_t local, uint32_t *bufa, uint32_t *bufb,
                                          uint32_t *tws) {
    const int k1 = J.k1, k2 = J.k2, k = k1 + k2;
    const int gl = k - 12;  // log2 of the blocks of one prime: N / NTT_ROWS_BLOCK
    constexpr int q = Q;
    const int64_t base = (local & (((int64_t)1 << gl) - 1)) * NTT_ROWS_BLOCK;  // whole rows, contiguous
    constexpr NttPrime P = ntt_prime_c(Q);
    uint32_t *x = J.x + ((int64_t)q << k) + base;
    const uint32_t *y = J.y + ((int64_t)q << k) + base;
    const int t = threadIdx.x, tp = pad_ix(t);
    // both directions' stage twiddles, loaded with the first residues (the inverse ones wait in
    // registers until the forward transforms are done)
    constexpr int TPT = TWS / NTT_TPB;
    uint32_t twf[TPT], twi[TPT];
#pragma unroll
    for (int m = 0; m < TPT; ++m) {
        twf[m] = ldg(&ntt_stage_tab[q][0][t + m * NTT_TPB]);
        twi[m] = ldg(&ntt_stage_tab[q][1][t + m * NTT_TPB]);
    }
    // Rows of 2^9 and more: the outermost pass of each direction runs in registers, on the
    // residues as they come from HBM (forward) and as they go back (inverse), which saves an
    // LDS round trip and a barrier each way
    const bool regs = k2 >= 9 && (k2 <= 10 || TPT >= 16);
    static_assert(EPT_R == CH, "a thread's residues of one operand in one round of loads");
    {
        uint32_t u[EPT_R], v[EPT_R];
#pragma unroll
        for (int i = 0; i < EPT_R; ++i) {
            u[i] = ldg(x + t + i * NTT_TPB);
            v[i] = ldg(y + t + i * NTT_TPB);
        }
        if (regs) {
            row_outer<false>(k2, u, twf, P);
            row_outer<false>(k2, v, twf, P);
        }
#pragma unroll
        for (int i = 0; i < EPT_R; ++i) {
            bufa[tp + i * PSTEP] = u[i];
            bufb[tp + i * PSTEP] = v[i];
        }
    }
#pragma unroll
    for (int m = 0; m < TPT; ++m) tws[t + m * NTT_TPB] = twf[m];
    __syncthreads();
    if (regs)  // both operands
        lds_transform_pad_any<false, NTT_ROWS_BLOCK, 0, false, 2, false>(k2, bufa, tws, P, bufb);
    else
        lds_transform_pad_any<false, NTT_ROWS_BLOCK, 0, false, 2>(k2, bufa, tws, P, bufb);
    // pointwise A B R^-1 (equal positions: both in the order the forward steps left; A, B < 2P,
    // so A B < P 2^32 and the product is below 2P), then the inverse twiddles replace the
    // forward ones (every thread is past the forward transforms' barrier)
#pragma unroll 4
    for (int i = 0; i < EPT_R; ++i) {
        const int e = tp + i * PSTEP;
        bufa[e] = mmul_lazy(bufa[e], bufb[e], P);
    }
#pragma unroll
    for (int m = 0; m < TPT; ++m) tws[t + m * NTT_TPB] = twi[m];
    __syncthreads();
    // out as they are (below 4P): the inverse columns apply the inverse twiddles as they read
    // them back (the scale 1 / N came in with the second operand's forward twiddles)
    if (regs) {
        lds_transform_pad_any<true, NTT_ROWS_BLOCK, 0, false, 1, false>(k2, bufa, tws, P);
        uint32_t u[EPT_R];
#pragma unroll
        for (int i = 0; i < EPT_R; ++i) u[i] = bufa[tp + i * PSTEP];
        row_outer<true>(k2, u, twi, P);
#pragma unroll
        for (int i = 0; i < EPT_R; ++i) stg(x + t + i * NTT_TPB, u[i]);
    } else {
        lds_transform_pad_any<true, NTT_ROWS_BLOCK, 0>(k2, bufa, tws, P);
#pragma unroll 8
        for (int i = 0; i < EPT_R; ++i) stg(x + t + i * NTT_TPB, bufa[tp + i * PSTEP]);
    }
}

// TWS: words of stage twiddles, 2^k2 (rows of up to 2^10 take 38 KB of LDS and four blocks fit
// on a CU; longer rows take the larger table and three blocks)
template <int TWS>
__global__ __launch_bounds__(NTT_TPB) void ntt_rows_kernel(Launch<NttJob> L) {
    __shared__ uint32_t bufa[pad_len(NTT_ROWS_BLOCK)];
    __shared__ uint32_t bufb[pad_len(NTT_ROWS_BLOCK)];
    __shared__ uint32_t tws[TWS];
    int64_t local;
    const NttJob J = get_job(L, (int64_t)blockIdx.x, local);
    if ((local >> (J.k1 + J.k2 - 12)) == 0)
        rows_body<0, TWS>(J, local, bufa, bufb, tws);
    else
        rows_body<1, TWS>(J, local, bufa, bufb, tws);
}
constexpr int NTT_ROWS_TWS_SMALL = 1 << 10, NTT_ROWS_TWS = 1 << 12;
static_assert(NTT_ROWS_TWS >= (1 << (NTT_MAX_LOG - NTT_MAX_LOG / 2)), "stage twiddles of the longest rows");

template <int Q, int TWS>
__device__ __forceinline__ void inv_cols_body(const NttJob &J, int64_t local, uint32_t *buf, uint32_t *tws) {
    const int k1 = J.k1, k2 = J.k2, k = k1 + k2;
    const int lc = 13 - k1, C = 1 << lc, SC = pad_len(1 << k1) + 1;
    const int gl = k - 13;
    constexpr int q = Q;
    const int64_t c0 = (local & (((int64_t)1 << gl) - 1)) * C;
    constexpr NttPrime P = ntt_prime_c(Q);
    uint32_t *x = J.x + ((int64_t)q << k);
    const int t = threadIdx.x;
    constexpr int TPT = TWS / NTT_TPB;
    uint32_t twi[TPT];
#pragma unroll
    for (int m = 0; m < TPT; ++m) twi[m] = ldg(&ntt_stage_tab[q][1][t + m * NTT_TPB]);
    // element e = t + 256 i: column c = t mod C, row n1 = t / C + i 256 / C
    const int ct = t & (C - 1), n1t = t >> lc, n1s = NTT_TPB >> lc;
    uint32_t *bt = buf + ct * SC;
    // The inverse twiddle of row n1, column n2 is w_N^-(n2 bitrev_k1(n1)).  With n1s = 2^(k1 - 5)
    // and i < 32, bitrev_k1(n1t + i n1s) = 32 bitrev_(k1-5)(n1t) + bitrev_5(i), so a thread's
    // twiddles are A g^j (A = w_N^-(32 n2 bitrev(n1t)), g = w_N^-n2, j = bitrev_5(i)): the even j
    // (i < 16) first, then the odd ones, each run of 16 by a recurrence in g^2.  Inputs below 4P,
    // twiddles fully reduced: the products stay below 2P.
    static_assert(EPT == 32 && CH == 16, "two runs of 16 twiddles per thread");
    const int sh = NTT_ROOT_LOG - k;
    const uint32_t emask = (1u << NTT_ROOT_LOG) - 1u, n2 = (uint32_t)(c0 + ct);
    const uint32_t g = root_pow(q, (0u - (n2 << sh)) & emask, P);
    const uint32_t g2 = mmul(g, g, P);
    uint32_t a0 = root_pow(q, (0u - (((n2 * bitrev((uint32_t)n1t, k1 - 5)) << 5) << sh)) & emask, P);
#pragma unroll 1
    for (int i0 = 0; i0 < EPT; i0 += CH) {
        uint32_t v[CH], tw[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) v[i] = ldg(x + ((int64_t)(n1t + (i0 + i) * n1s) << k2) + c0 + ct);
        tw[0] = a0;  // A g^(i0 / 16)
#pragma unroll
        for (int m = 1; m < CH; ++m) tw[m] = mmul(tw[m - 1], g2, P);
#pragma unroll
        for (int i = 0; i < CH; ++i) bt[pad_ix(n1t + (i0 + i) * n1s)] = mmul_lazy(v[i], tw[bitrev((uint32_t)i, 4)], P);
        a0 = mmul(a0, g, P);
    }
#pragma unroll
    for (int m = 0; m < TPT; ++m) tws[t + m * NTT_TPB] = twi[m];
    __syncthreads();
    lds_transform_pad_any<true, NTT_BLOCK, 1>(k1, buf, tws, P);
    // the residues of terms N2 n1 + n2 in natural order, fully reduced, in place (the block's
    // columns hold exactly the positions it read)
#pragma unroll 8
    for (int i = 0; i < EPT; ++i) {
        const int n1 = n1t + i * n1s;
        stg(x + ((int64_t)n1 << k2) + c0 + ct, red1(red2(bt[pad_ix(n1)], P.p), P.p));
    }
}

template <int TWS>
__global__ __launch_bounds__(NTT_TPB) void ntt_inv_cols_kernel(Launch<NttJob> L) {
    __shared__ uint32_t buf[NTT_COL_BUF];
    __shared__ uint32_t tws[TWS];
    int64_t local;
    const NttJob J = get_job(L, xcd_block((int64_t)blockIdx.x, L.total_blocks), local);
    if ((local >> (J.k1 + J.k2 - 13)) == 0)
        inv_cols_body<0, TWS>(J, local, buf, tws);
    else
        inv_cols_body<1, TWS>(J, local, buf, tws);
}

// the join: one thread per limb column, the (at most two for w >= 16, three for w >= 11) terms
// whose bit weight falls in it
__global__ __launch_bounds__(NTT_TPB) void ntt_join_kernel(Launch<NttJoinJob> L) {
    int64_t local;
    NttJoinJob J = find_job(L, (int64_t)blockIdx.x, local);
    J.x = at(L.base_ws, J.x);
    J.cols = at(L.base_ws, J.cols);
    const int64_t col = local * NTT_TPB + threadIdx.x;
    if (col >= J.ncols) return;
    // bit positions fit in 32 bits (a product has at most 30 2^23 < 2^28 bits): one 32-bit
    // division finds the column's first term, the rest follow by adding w
    const uint32_t w = (uint32_t)J.w, b0 = 32u * (uint32_t)col, nz = (uint32_t)J.nz;
    uint32_t m = (b0 + w - 1u) / w;  // first term with w m >= 32 col
    uint64_t lo = 0;
    uint32_t hi = 0;
    for (uint32_t bit = m * w; bit < b0 + 32u && m < nz; ++m, bit += w) {
        const uint64_t z = crt2(ldg(J.x + m), ldg(J.x + J.n + m));
        const int sh = (int)(bit - b0);  // 0 .. 31
        const uint64_t zl = z << sh;
        const uint32_t zh = sh ? (uint32_t)(z >> (64 - sh)) : 0u;
        lo += zl;
        hi += zh + (lo < zl ? 1u : 0u);
    }
    uint32_t v[3] = {(uint32_t)lo, (uint32_t)(lo >> 32), hi};
    stg_words<3>(J.cols + 3 * col, v);
}

// ---- host side -----------------------------------------------------------------------------------

static uint64_t mulmod_h(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((unsigned __int128)a * b % p); }
static uint64_t powmod_h(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1;
    for (a %= p; e; e >>= 1, a = mulmod_h(a, a, p))
        if (e & 1) r = mulmod_h(r, a, p);
    return r;
}

uint32_t ntt_scale(int q, int k) {
    const uint64_t p = q == 0 ? NTT_P0 : NTT_P1;
    const uint64_t r2 = powmod_h(2, 64, p);                // R^2
    const uint64_t ninv = powmod_h((p + 1) / 2, (uint64_t)k, p);  // 2^-k
    return (uint32_t)mulmod_h(r2, ninv, p);
}

bool ntt_shape(int64_t na, int64_t nb, int min_log, int &k1, int &k2, int &w, int64_t &npa, int64_t &npb) {
    for (int k = std::max(min_log, NTT_MIN_LOG); k <= NTT_MAX_LOG; ++k) {
        const int64_t N = (int64_t)1 << k;
        for (int ww = 1; ww <= 30; ++ww) {
            const int64_t pa = cdiv(32 * na, ww), pb = cdiv(32 * nb, ww);
            if (pa + pb - 1 > N) continue;
            // exact: every term below min(pa, pb) 2^(2w) <= 2^59 < P0 P1
            if (2 * ww + ceil_log2(std::min(pa, pb)) > 59) break;
            // rows as long as the small stage table allows (2^10), columns at most 2^11 and at
            // least 2^6: the row step costs less per transform stage than the column steps
            k2 = std::min(std::max(10, k - 11), k - 6);
            k1 = k - k2;
            w = ww;
            npa = pa;
            npb = pb;
            return true;
        }
    }
    return false;
}

int ntt_prepare() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KS_EHIP;
    std::lock_guard<std::mutex> lk(mu);
    if (done[dev]) return KS_OK;
    static uint32_t host[2][2][NTT_TAB];
    const uint64_t prime[2] = {NTT_P0, NTT_P1}, gen[2] = {3, 3};  // primitive roots
    for (int q = 0; q < 2; ++q) {
        const uint64_t p = prime[q];
        const uint64_t w = powmod_h(gen[q], (p - 1) >> NTT_ROOT_LOG, p);  // order 2^23
        const uint64_t R = ((uint64_t)1 << 32) % p;
        const uint64_t wh = powmod_h(w, NTT_TAB, p);
        uint64_t a = 1, b = 1;
        for (int i = 0; i < NTT_TAB; ++i) {
            host[q][0][i] = (uint32_t)mulmod_h(a, R, p);
            host[q][1][i] = (uint32_t)mulmod_h(b, R, p);
            a = mulmod_h(a, wh, p);
            b = mulmod_h(b, w, p);
        }
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(ntt_tab), host, sizeof(host), 0, hipMemcpyHostToDevice) != hipSuccess)
        return KS_EHIP;
    static uint32_t stage[2][2][NTT_STAGE_TW];
    for (int q = 0; q < 2; ++q) {
        const uint64_t p = prime[q];
        const uint64_t w = powmod_h(gen[q], (p - 1) >> NTT_ROOT_LOG, p);
        const uint64_t R = ((uint64_t)1 << 32) % p;
        stage[q][0][0] = stage[q][1][0] = 0;
        for (int i = 1; i < NTT_STAGE_TW; ++i) {
            int sl = 0;
            while ((2 << sl) <= i) ++sl;  // half-size 2^sl <= i < 2^(sl+1)
            const uint64_t e = (uint64_t)(i - (1 << sl)) << (NTT_ROOT_LOG - 1 - sl);  // w_(2h)^j = w^e
            const uint64_t ei = (((uint64_t)1 << NTT_ROOT_LOG) - e) & (((uint64_t)1 << NTT_ROOT_LOG) - 1);
            stage[q][0][i] = (uint32_t)mulmod_h(powmod_h(w, e, p), R, p);
            stage[q][1][i] = (uint32_t)mulmod_h(powmod_h(w, ei, p), R, p);
        }
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(ntt_stage_tab), stage, sizeof(stage), 0, hipMemcpyHostToDevice) != hipSuccess)
        return KS_EHIP;
    done[dev] = true;
    return KS_OK;
}

hipError_t launch_ntt_join(const Launch<NttJoinJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    ks_launch(ntt_join_kernel, dim3((unsigned)L.total_blocks), dim3(NTT_TPB), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_ntt_stage(int stage, const Launch<NttJob> &L, int max_k1, int max_k2, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    const dim3 g((unsigned)L.total_blocks), b(NTT_TPB);
    switch (stage) {
        case 0:
            if (max_k1 <= 10)
                ks_launch(ntt_fwd_cols_kernel<NTT_COLS_TWS_SMALL>, g, b, 0, s, L);
            else
                ks_launch(ntt_fwd_cols_kernel<NTT_COLS_TWS>, g, b, 0, s, L);
            break;
        case 1:
            if (max_k2 <= 10)
                ks_launch(ntt_rows_kernel<NTT_ROWS_TWS_SMALL>, g, b, 0, s, L);
            else
                ks_launch(ntt_rows_kernel<NTT_ROWS_TWS>, g, b, 0, s, L);
            break;
        case 2:
            if (max_k1 <= 10)
                ks_launch(ntt_inv_cols_kernel<NTT_COLS_TWS_SMALL>, g, b, 0, s, L);
            else
                ks_launch(ntt_inv_cols_kernel<NTT_COLS_TWS>, g, b, 0, s, L);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ks
