// ks_finish.hip -- reading the coefficients of h back off the recombined products.
//
// extract_kernel  KS1 (paper Section 3.1) and NEG2 (Section 3.3): coefficient k sits alone
//                 in slot k of the normalised value (slot width N, or 2N for the even and
//                 odd parts of the negated variant).  One thread per coefficient.
// anchor_kernel   Exact h_k at the first coefficient before each chain segment (below).
// chain_kernel    KS4 (Section 3.4): the carry-aware reconstruction of Section 3.2, run on
//                 the even part and on the odd part at base Y = 2^(2N); RECIP2 (Section
//                 3.2): the same reconstruction once at base 2^N.  It leaves alpha_k and
//                 beta_k (h_k + C = alpha_k + Y beta_k) in scratch.
// finish_kernel   One thread per coefficient: h_k from alpha_k, beta_k, written out.
//
// Section 3.2's procedure is one sequential chain over all coefficients.  It carries, from
// coefficient k-1 to k, only the low half alpha_{k-1} and the carry sigma_{k-1} that the
// lower coefficients push into digit k of A = h(Y).  Both follow from the exact value of
// h_{k-1}:  alpha_{k-1} = h_{k-1} mod Y,  sigma_{k-1} = floor(h_{k-1} / Y) + [u_{k-1} <
// alpha_{k-1}].  So the chain is cut into segments of K coefficients and every segment but
// the first starts from an anchor h_{sK-1} computed directly as a dot product of the inputs;
// segments then run in parallel, one per lane.  The last value each segment produces is the
// next segment's anchor, and the final coefficient satisfies the two relations the procedure
// leaves unused (alpha_{m-1} = w_m, sigma_{m-1} = u_m): all three are checked on the device.
//
// Signed inputs: every slot holds h_k + C with C = 2^off_bit, removed on output.
#include "ks_anchor.h"
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

// ---- (r 2^32 + word) mod p, r < p < 2^62 ------------------------------------------------------
// Quotient estimated in double precision from a reciprocal pinv = 1/p computed once, then
// corrected exactly in 64-bit integers (the floating-point reduction technique used by Shoup's
// NTL): q < 2^32 and the estimate's relative error is a few units in 2^-53, so it is off by
// at most one.
__device__ __forceinline__ uint64_t mod_step(uint64_t r, uint32_t word, uint64_t p, double pinv) {
    const uint64_t x = (r << 32) | word;
    if ((p >> 32) == 0) return x % p;  // r < 2^32 here, so x is exact
    const double xd = (double)r * 4294967296.0 + (double)word;
    const uint64_t q = (uint64_t)(xd * pinv);
    uint64_t d = x - q * p;             // x - q p in [-p, 2p), modulo 2^64
    if ((int64_t)d < 0) d += p;
    while (d >= p) d -= p;
    return d;
}

// ---- extraction ------------------------------------------------------------------------------

__global__ __launch_bounds__(EXTRACT_TPB) void extract_kernel(Launch<ExtractJob> L) {
    int64_t local;
    const ExtractJob J = get_job(L, (int64_t)blockIdx.x, local);
    const int64_t k = local * EXTRACT_TPB + threadIdx.x;
    if (k >= J.count) return;
    const int64_t s0 = k * J.slot;
    const int64_t idx = J.out_first + k * J.out_step;
    if (J.mod_p == 0) {
        uint32_t *o = J.out + idx * J.w_out;
        uint32_t borrow = 0;
        for (int t = 0; t < J.w_out; ++t) {
            const int64_t bit = 32 * (int64_t)t;
            uint32_t word = 0;
            if (bit < J.slot) {
                word = bits_word(J.src, J.n_src, s0 + bit);
                if (J.slot - bit < 32) word &= (1u << (J.slot - bit)) - 1u;
            }
            uint32_t sub = (J.off_bit >= 0 && (J.off_bit >> 5) == t) ? (1u << (J.off_bit & 31)) : 0u;
            uint64_t d = (uint64_t)word - sub - borrow;
            o[t] = (uint32_t)d;
            borrow = (uint32_t)(d >> 63) & 1u;
        }
    } else {
        const int nl = (int)((J.slot + 31) >> 5);
        const double pinv = 1.0 / (double)J.mod_p;
        uint64_t r = 0;
        for (int t = nl - 1; t >= 0; --t) {
            const int64_t bit = 32 * (int64_t)t;
            uint32_t word = bits_word(J.src, J.n_src, s0 + bit);
            if (J.slot - bit < 32) word &= (1u << (J.slot - bit)) - 1u;
            r = mod_step(r, word, J.mod_p, pinv);
        }
        reinterpret_cast<uint64_t *>(J.out)[idx] = r;
    }
}

// ---- anchors -----------------------------------------------------------------------------------

template <int W>
__global__ __launch_bounds__(ANCHOR_TPB) void anchor_kernel(Launch<AnchorJob> L) {
    int64_t local;
    const AnchorJob J = get_job(L, xcd_block((int64_t)blockIdx.x, L.total_blocks), local);
    if (J.nseg2 > 0)
        anchor_pair_block<W>(J, local);
    else
        anchor_block<W>(J, local);
}

// ---- chains ------------------------------------------------------------------------------------

template <int NW>
struct MW {
    uint32_t w[NW];
};

// Nd-bit digit starting at bit0 of an n-limb array
template <int NW>
__device__ __forceinline__ MW<NW> read_digit(const uint32_t *x, int64_t n, int64_t bit0, int Nd) {
    MW<NW> d;
    const int64_t q = bit0 >> 5;
    const int o = (int)(bit0 & 31);
    uint32_t l[NW + 1];
#pragma unroll
    for (int t = 0; t <= NW; ++t) {
        const bool ok = q + t >= 0 && q + t < n;
        const uint32_t v = ldg(x + (ok ? q + t : 0));
        l[t] = ok ? v : 0u;
    }
#pragma unroll
    for (int t = 0; t < NW; ++t) d.w[t] = o ? (l[t] >> o) | (l[t + 1] << (32 - o)) : l[t];
    const int tb = Nd - 32 * (NW - 1);
    if (tb < 32) d.w[NW - 1] &= (1u << tb) - 1u;
    return d;
}

// The NW + 1 words that hold an Nd-bit digit at bit0, loaded as they are (clamped addresses, no
// branches, global rather than flat loads), so that a ring of them stays in flight; words
// outside [0, n) are zeroed only where the digit is formed from them.
template <int NW>
struct RawDigit {
    uint32_t l[NW + 1];
};

template <int NW>
__device__ __forceinline__ void load_raw(RawDigit<NW> &r, const uint32_t *x, int64_t n, int64_t bit0) {
    const int64_t q = bit0 >> 5;
    if (q >= 0 && q + NW < n) {  // the usual case: one vector load (lanes of a wave read far apart)
        ldg_words<NW + 1>(x + q, r.l);
        return;
    }
#pragma unroll
    for (int t = 0; t <= NW; ++t) {
        const bool ok = q + t >= 0 && q + t < n;
        r.l[t] = ldg(x + (ok ? q + t : 0));
    }
}

template <int NW>
__device__ __forceinline__ MW<NW> raw_digit(const RawDigit<NW> &r, int64_t n, int64_t bit0, int Nd) {
    MW<NW> d;
    const int64_t q = bit0 >> 5;
    const int o = (int)(bit0 & 31);
    uint32_t l[NW + 1];
#pragma unroll
    for (int t = 0; t <= NW; ++t) l[t] = (q + t >= 0 && q + t < n) ? r.l[t] : 0u;
#pragma unroll
    for (int t = 0; t < NW; ++t) d.w[t] = o ? (l[t] >> o) | (l[t + 1] << (32 - o)) : l[t];
    const int tb = Nd - 32 * (NW - 1);
    if (tb < 32) d.w[NW - 1] &= (1u << tb) - 1u;
    return d;
}

template <int NW>
__device__ __forceinline__ MW<NW> sub_mod(const MW<NW> &a, const MW<NW> &b, uint32_t extra, int Nd) {
    MW<NW> r;
    uint64_t br = extra;
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        uint64_t d = (uint64_t)a.w[t] - b.w[t] - br;
        r.w[t] = (uint32_t)d;
        br = (d >> 63) & 1u;
    }
    const int tb = Nd - 32 * (NW - 1);
    if (tb < 32) r.w[NW - 1] &= (1u << tb) - 1u;
    return r;
}

template <int NW>
__device__ __forceinline__ bool mw_lt(const MW<NW> &a, const MW<NW> &b) {
    bool lt = false, decided = false;
#pragma unroll
    for (int t = NW - 1; t >= 0; --t) {
        if (!decided && a.w[t] != b.w[t]) {
            lt = a.w[t] < b.w[t];
            decided = true;
        }
    }
    return lt;
}

template <int NW>
__device__ __forceinline__ bool mw_eq(const MW<NW> &a, const MW<NW> &b) {
    bool eq = true;
#pragma unroll
    for (int t = 0; t < NW; ++t) eq = eq && (a.w[t] == b.w[t]);
    return eq;
}

template <int NW>
__device__ __forceinline__ MW<NW> add_bit(const MW<NW> &a, uint32_t c) {
    MW<NW> r;
    uint64_t cc = c;
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        uint64_t s = (uint64_t)a.w[t] + cc;
        r.w[t] = (uint32_t)s;
        cc = s >> 32;
    }
    return r;
}

template <int NW>
__device__ __forceinline__ uint32_t mw_word(const MW<NW> &a, int64_t idx) {
    uint32_t r = 0;
#pragma unroll
    for (int t = 0; t < NW; ++t) r = (idx == t) ? a.w[t] : r;
    return r;
}

// bits [p, p+32) of the Nd-bit digit a (zero outside [0, Nd))
template <int NW>
__device__ __forceinline__ uint32_t mw_bits(const MW<NW> &a, int64_t p) {
    if (p <= -32) return 0u;
    if (p < 0) return mw_word(a, 0) << (int)(-p);
    const int64_t q = p >> 5;
    const int o = (int)(p & 31);
    uint32_t lo = mw_word(a, q);
    if (o == 0) return lo;
    return (lo >> o) | (mw_word(a, q + 1) << (32 - o));
}

// limb t of h' = alpha + 2^Nd beta
template <int NW>
__device__ __forceinline__ uint32_t hword(const MW<NW> &al, const MW<NW> &be, int Nd, int t) {
    return mw_bits(al, 32 * (int64_t)t) | mw_bits(be, 32 * (int64_t)t - Nd);
}

// all limbs of h' = alpha + 2^Nd beta (alpha, beta < 2^Nd), in a register array
template <int NW>
__device__ __forceinline__ void hprime(const MW<NW> &al, const MW<NW> &be, int Nd, uint32_t (&H)[2 * NW + 1]) {
    const int q = Nd >> 5, o = Nd & 31;
#pragma unroll
    for (int t = 0; t < 2 * NW + 1; ++t) {
        uint32_t v = t < NW ? al.w[t] : 0u;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            if (t == i + q) v |= be.w[i] << o;
            if (o && t == i + q + 1) v |= be.w[i] >> (32 - o);
        }
        H[t] = v;
    }
}

// One lane per segment.  Digits are read straight from the recombined products through a
// ring of CHAIN_P(NW) prefetched steps: a step takes its digits from the ring and at once
// issues the loads of the step CHAIN_P later, so the chain's dependent arithmetic overlaps
// the memory latency of the steps ahead.  The lanes of a wave read far-apart segments, and
// a wave runs alone on its SIMD, so registers are plentiful: 16 steps in flight (digits of up
// to 3 words) took the 64-product modular batch's chains from 164 to 154 us against 8.
template <int NW>
struct ChainRing {
    static constexpr int P = NW <= 3 ? 16 : (NW <= 5 ? 8 : 4);
};

// Segment s of chain J on this lane.  ROUNDS: whole rounds of P steps without guards, then the
// last partial round (the same loads in flight on every path, so the waits stay partial:
// long segments); else one guarded loop (half the code: short segments, where instruction
// fetch is a large part of the time).
template <int NW, bool ROUNDS>
__device__ __forceinline__ void chain_seg(const ChainJob &J, int64_t s, uint32_t *devstat) {
    constexpr int P = ChainRing<NW>::P;
    if (s >= J.nseg) return;
    const int Nd = J.Nd;
    const int64_t m = J.m;
    const int64_t k0 = s * J.K;
    int64_t k1 = k0 + J.K;
    if (k1 > m) k1 = m;
    const int hw = (2 * Nd + 31) >> 5;  // limbs of h' = alpha + Y beta
#define U_DIGIT(c) read_digit<NW>(J.A, J.nA, (c) * (int64_t)Nd, Nd)
#define W_DIGIT(c) read_digit<NW>(J.B, J.nB, (m - (c)) * (int64_t)Nd, Nd)

    MW<NW> sigma, aprev;
#pragma unroll
    for (int t = 0; t < NW; ++t) { sigma.w[t] = 0; aprev.w[t] = 0; }
    if (s > 0) {
        const uint32_t *anc = J.anchors + s * J.aw;
        MW<NW> al = read_digit<NW>(anc, J.aw, 0, Nd);
        MW<NW> be = read_digit<NW>(anc, J.aw, Nd, Nd);
        MW<NW> u = U_DIGIT(k0 - 1);
        aprev = al;
        sigma = add_bit(be, mw_lt(u, al) ? 1u : 0u);
    }
    MW<NW> wc = W_DIGIT(k0);
    MW<NW> alpha = aprev, beta;
    // ring slot j holds the digits u_c and w_{c+1} of the steps c = j (mod P)
    RawDigit<NW> ru[P], rw[P];
    // ROUNDS: a refill past the segment's last step re-reads the first step's words (cached,
    // unused), so the refill needs no branch; else refills past the last step are skipped
    auto fetch = [&](int j, int64_t c) {
        if (!ROUNDS && c >= k1) return;
        const int64_t cc = c < k1 ? c : k0;
        load_raw(ru[j], J.A, J.nA, cc * (int64_t)Nd);
        load_raw(rw[j], J.B, J.nB, (m - (cc + 1)) * (int64_t)Nd);
    };
    // step c: digits from ring slot j, which is refilled with step c + P's; alpha_c and beta_c
    // (for the finishing pass) go to ab[j] -- in whole rounds they are stored after the round,
    // behind the round's refills: memory operations complete in order for the wait counter, so
    // a store issued between a refill and its use would put the store's latency on every step
    uint32_t ab[P][2 * NW];
    auto step = [&](int j, int64_t c) {
        const MW<NW> u = raw_digit(ru[j], J.nA, c * (int64_t)Nd, Nd);
        const MW<NW> wn = raw_digit(rw[j], J.nB, (m - (c + 1)) * (int64_t)Nd, Nd);
        fetch(j, c + P);
        __builtin_amdgcn_sched_barrier(0);
        alpha = sub_mod(u, sigma, 0u, Nd);          // alpha_c = u_c - sigma_{c-1}  (mod Y)
        uint32_t delta = mw_lt(u, sigma) ? 1u : 0u;  // carry of the low half into digit c+1
        uint32_t eps = mw_lt(wn, alpha) ? 1u : 0u;   // eps_c = [alpha_c > w_{c+1}]
        beta = sub_mod(wc, aprev, eps, Nd);          // beta_c = w_c - alpha_{c-1} - eps_c (mod Y)
        sigma = add_bit(beta, delta);                // sigma_c = beta_c + delta
        aprev = alpha;
        wc = wn;
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            ab[j][t] = alpha.w[t];
            ab[j][NW + t] = beta.w[t];
        }
    };
#pragma unroll
    for (int j = 0; j < P; ++j) fetch(j, k0 + j);
    int64_t cb = k0;
    if (ROUNDS) {
        for (; cb + P <= k1; cb += P) {
#pragma unroll
            for (int j = 0; j < P; ++j) step(j, cb + j);
            // the round's P (alpha, beta) pairs are contiguous: wide stores
            stg_words<2 * NW * P>(J.hbuf + cb * (2 * NW), &ab[0][0]);
        }
    }
    for (; cb < k1; cb += P) {
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (cb + j < k1) {
                step(j, cb + j);
                stg_words<2 * NW>(J.hbuf + (cb + j) * (2 * NW), ab[j]);
            }
    }
    // self-checks: the segment ends on the next anchor; the chain ends on the two unused relations
    bool ok = true;
    if (k1 < m) {
        const uint32_t *anc = J.anchors + (s + 1) * J.aw;
        for (int t = 0; t < J.aw; ++t) ok = ok && (anc[t] == (t < hw ? hword(alpha, beta, Nd, t) : 0u));
    } else if (k1 > k0) {
        ok = mw_eq(alpha, W_DIGIT(m)) && mw_eq(sigma, U_DIGIT(m));
    }
    if (!ok) set_status(devstat, KS_DEVSTAT_CHECK);
#undef U_DIGIT
#undef W_DIGIT
}

// ---- the chain's fast path ----------------------------------------------------------------------
//
// When every digit a segment reads lies inside A and B (the recombined products hold
// ceil((m + 1) Nd / 32) + 1 limbs, which covers the NW + 1 words of digit m - 1 once Nd >= 16) and
// the bit offsets fit in 32 bits, a step needs no bounds checks: a digit is NW funnel shifts
// of the NW + 1 words one vector load brought in, and the chain's state is (beta, delta) rather
// than sigma = beta + delta, so that alpha = (u - beta - delta) mod Y and delta' = [u < sigma]
// come out of one subtraction with borrow.
template <int NW>
__device__ __forceinline__ bool chain_fast_ok(const ChainJob &J) {
    const int64_t top = (((J.m - 1) * (int64_t)J.Nd) >> 5) + NW;
    return J.Nd >= 16 && J.m >= 1 && (J.m + 1) * (int64_t)J.Nd < ((int64_t)1 << 31) && top < J.nA &&
           top < J.nB;
}

// a - b - bin over NW words into r; returns the borrow out, [a < b + bin] (a chain of
// subtractions with borrow, one instruction per word)
template <int NW>
__device__ __forceinline__ uint32_t mw_sub_borrow(const MW<NW> &a, const MW<NW> &b, uint32_t bin, MW<NW> &r) {
    unsigned int br = bin;
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        unsigned int bo;
        r.w[t] = __builtin_subc(a.w[t], b.w[t], br, &bo);
        br = bo;
    }
    return br;
}

template <int NW>
__device__ __forceinline__ MW<NW> funnel_digit(const uint32_t (&l)[NW + 1], uint32_t sh, uint32_t topmask) {
    MW<NW> d;
#pragma unroll
    for (int t = 0; t < NW; ++t) d.w[t] = __builtin_amdgcn_alignbit(l[t + 1], l[t], sh);
    d.w[NW - 1] &= topmask;
    return d;
}

template <int NW>
__device__ __forceinline__ void chain_seg_fast(const ChainJob &J, int64_t s, uint32_t *devstat) {
    constexpr int P = ChainRing<NW>::P;
    if (s >= J.nseg) return;
    const uint32_t Nd = (uint32_t)J.Nd;
    const int64_t m = J.m;
    const int64_t k0 = s * J.K;
    const int64_t k1 = k0 + J.K < m ? k0 + J.K : m;
    const int hw = (int)((2 * Nd + 31) >> 5);
    const uint32_t tb = Nd - 32u * (NW - 1);
    const uint32_t topmask = tb >= 32 ? 0xffffffffu : (1u << tb) - 1u;
    const uint32_t mm1 = (uint32_t)(m - 1), last = (uint32_t)(k1 - 1), k1u = (uint32_t)k1;
    MW<NW> beta, aprev, wc;
    bool dl = false;  // a lane mask, so it feeds the next step's borrow chain directly
#pragma unroll
    for (int t = 0; t < NW; ++t) { beta.w[t] = 0; aprev.w[t] = 0; }
    if (s > 0) {
        const uint32_t *anc = J.anchors + s * J.aw;
        const MW<NW> al = read_digit<NW>(anc, J.aw, 0, (int)Nd);
        beta = read_digit<NW>(anc, J.aw, Nd, (int)Nd);
        const MW<NW> u = read_digit<NW>(J.A, J.nA, (k0 - 1) * (int64_t)Nd, (int)Nd);
        aprev = al;
        MW<NW> scratch;
        dl = mw_sub_borrow(u, al, 0u, scratch) != 0;  // [u < al]: sigma = beta + dl
    }
    wc = read_digit<NW>(J.B, J.nB, (m - k0) * (int64_t)Nd, (int)Nd);
    MW<NW> alpha = aprev;
    uint32_t ru[P][NW + 1], rw[P][NW + 1], su[P], sw[P];
    // step c's words (clamped to the segment's last step: a refill past it reads words that stay
    // unused); B's digit of step c is w_{c+1}, at m - c - 1.  Steps, bit offsets and byte
    // offsets fit in 32 bits ((m + 1) Nd < 2^31): the loads take a scalar base and a vector offset
    auto fetch = [&](int j, uint32_t c) {
        const uint32_t cc = c < k1u ? c : last;
        const uint32_t ou = cc * Nd, ow = (mm1 - cc) * Nd;
        ldg_words<NW + 1>(byte_at(J.A, (ou >> 5) << 2), ru[j]);
        ldg_words<NW + 1>(byte_at(J.B, (ow >> 5) << 2), rw[j]);
        su[j] = ou & 31u;
        sw[j] = ow & 31u;
    };
    uint32_t ab[P][2 * NW];
    auto step = [&](int j, uint32_t c) {
        const MW<NW> u = funnel_digit<NW>(ru[j], su[j], topmask);
        const MW<NW> wn = funnel_digit<NW>(rw[j], sw[j], topmask);
        fetch(j, c + P);
        __builtin_amdgcn_sched_barrier(0);
        dl = mw_sub_borrow(u, beta, dl ? 1u : 0u, alpha) != 0;  // alpha_c = u_c - sigma_{c-1}, delta_c
        alpha.w[NW - 1] &= topmask;
        MW<NW> scratch;
        const uint32_t eps = mw_sub_borrow(wn, alpha, 0u, scratch);  // [w_{c+1} < alpha_c]
        // the differences are kept (empty uses, no instruction): otherwise the borrow is
        // rewritten as a compare tree combined on the scalar unit, whose round trips sit in
        // the chain's dependent path; kept, it is NW subtractions with borrow
#pragma unroll
        for (int t = 0; t < NW; ++t) asm volatile("" ::"v"(scratch.w[t]));
        mw_sub_borrow(wc, aprev, eps, beta);                         // beta_c = w_c - alpha_{c-1} - eps_c
        beta.w[NW - 1] &= topmask;
        aprev = alpha;
        wc = wn;
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            ab[j][t] = alpha.w[t];
            ab[j][NW + t] = beta.w[t];
        }
    };
#pragma unroll
    for (int j = 0; j < P; ++j) fetch(j, (uint32_t)k0 + j);
    uint32_t cb = (uint32_t)k0;
    for (; cb + P <= k1u; cb += P) {
#pragma unroll
        for (int j = 0; j < P; ++j) step(j, cb + j);
        stg_words<2 * NW * P>(J.hbuf + (int64_t)cb * (2 * NW), &ab[0][0]);  // after the round's refills
    }
#pragma unroll
    for (int j = 0; j < P; ++j)
        if (cb + j < k1u) {
            step(j, cb + j);
            stg_words<2 * NW>(J.hbuf + (int64_t)(cb + j) * (2 * NW), ab[j]);
        }
    // self-checks, as in chain_seg
    bool ok = true;
    if (k1 < m) {
        const uint32_t *anc = J.anchors + (s + 1) * J.aw;
        for (int t = 0; t < J.aw; ++t) ok = ok && (anc[t] == (t < hw ? hword(alpha, beta, (int)Nd, t) : 0u));
    } else if (k1 > k0) {
        const MW<NW> sigma = add_bit(beta, dl ? 1u : 0u);
        ok = mw_eq(alpha, read_digit<NW>(J.B, J.nB, 0, (int)Nd)) &&
             mw_eq(sigma, read_digit<NW>(J.A, J.nA, m * (int64_t)Nd, (int)Nd));
    }
    if (!ok) set_status(devstat, KS_DEVSTAT_CHECK);
}

// A job's blocks of CHAIN_TPB lanes take its segments in order (single products).
template <int NW>
__global__ __launch_bounds__(CHAIN_TPB) void chain_kernel(Launch<ChainJob> L) {
    int64_t local;
    const ChainJob J = get_job(L, (int64_t)blockIdx.x, local);
    const int64_t s = local * CHAIN_TPB + threadIdx.x;
    if (s >= J.nseg) return;
    if (chain_fast_ok<NW>(J))
        chain_seg_fast<NW>(J, s, L.devstat);
    else
        chain_seg<NW, false>(J, s, L.devstat);
}

// Batches: the launch's units are segments, not blocks (a job's block0 and nblocks count its
// segments), and every lane looks up its own job, so the few segments of many small chains
// share waves.  NW = 0: the jobs have different digit widths (ascending in the table, so a
// wave mixes at most two) and each lane runs the body of its job's width.
template <int NW>
__global__ __launch_bounds__(CHAIN_TPB) void chain_lanes_kernel(Launch<ChainJob> L) {
    const int64_t g = (int64_t)blockIdx.x * CHAIN_TPB + threadIdx.x;
    if (g >= L.total_blocks) return;
    int64_t s;
    const ChainJob J = get_job(L, g, s);
    if constexpr (NW > 0) {
        if (chain_fast_ok<NW>(J))
            chain_seg_fast<NW>(J, s, L.devstat);
        else
            chain_seg<NW, true>(J, s, L.devstat);
    } else {
        switch ((J.Nd + 31) >> 5) {
#define KS_CHAIN_CASE(W)                        \
    case W:                                     \
        if (chain_fast_ok<W>(J))                \
            chain_seg_fast<W>(J, s, L.devstat); \
        else                                    \
            chain_seg<W, true>(J, s, L.devstat); \
        break;
            KS_CHAIN_CASE(1) KS_CHAIN_CASE(2) KS_CHAIN_CASE(3) KS_CHAIN_CASE(4) KS_CHAIN_CASE(5)
            KS_CHAIN_CASE(6) KS_CHAIN_CASE(7) KS_CHAIN_CASE(8) KS_CHAIN_CASE(9)
#undef KS_CHAIN_CASE
            default: break;
        }
    }
}

// One thread per coefficient c of a chain: h' = alpha_c + 2^Nd beta_c from the chain's scratch,
// written as h_{first + c step} = h' - C (w_out <= 2 NW + 1 limbs, since 2 Nd >= 2b + e) or as
// h' - C mod p.  Kept out of the chain, whose lanes are few and whose steps are dependent.
template <int NW>
__device__ __forceinline__ void finish_block(const ChainJob &J, int64_t local) {
    const int64_t c = local * FINISH_TPB + threadIdx.x;
    if (c >= J.m) return;
    const int Nd = J.Nd;
    MW<NW> alpha, beta;
    uint32_t ab[2 * NW];
    ldg_words<2 * NW>(J.hbuf + c * (2 * NW), ab);
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        alpha.w[t] = ab[t];
        beta.w[t] = ab[NW + t];
    }
    uint32_t H[2 * NW + 1];
    hprime(alpha, beta, Nd, H);
    const int64_t idx = J.out_first + c * J.out_step;
    if (J.mod_p == 0) {
        uint32_t *o = J.out + idx * J.w_out;
        uint32_t br = 0;
#pragma unroll
        for (int t = 0; t < 2 * NW + 1; ++t) {
            if (t < J.w_out) {
                const uint32_t sub = (J.off_bit >> 5) == t ? (1u << (J.off_bit & 31)) : 0u;
                const uint64_t d = (uint64_t)H[t] - (J.off_bit >= 0 ? sub : 0u) - br;
                o[t] = (uint32_t)d;
                br = (uint32_t)(d >> 63) & 1u;
            }
        }
    } else {
        // h' < 2^(2 Nd) and the slot constant is zero for residue inputs (unsigned)
        const int hw = (2 * Nd + 31) >> 5;
        const double pinv = 1.0 / (double)J.mod_p;
        uint64_t r = 0;
#pragma unroll
        for (int t = 2 * NW; t >= 0; --t)
            if (t < hw) r = mod_step(r, H[t], J.mod_p, pinv);
        reinterpret_cast<uint64_t *>(J.out)[idx] = r;
    }
}

template <int NW>
__global__ __launch_bounds__(FINISH_TPB) void finish_kernel(Launch<ChainJob> L) {
    int64_t local;
    const ChainJob J = get_job(L, (int64_t)blockIdx.x, local);
    finish_block<NW>(J, local);
}

__global__ __launch_bounds__(FINISH_TPB) void finish_any_kernel(Launch<ChainJob> L) {
    int64_t local;
    const ChainJob J = get_job(L, (int64_t)blockIdx.x, local);
    switch ((J.Nd + 31) >> 5) {
        case 1: finish_block<1>(J, local); break;
        case 2: finish_block<2>(J, local); break;
        case 3: finish_block<3>(J, local); break;
        case 4: finish_block<4>(J, local); break;
        case 5: finish_block<5>(J, local); break;
        case 6: finish_block<6>(J, local); break;
        case 7: finish_block<7>(J, local); break;
        case 8: finish_block<8>(J, local); break;
        case 9: finish_block<9>(J, local); break;
        default: break;
    }
}

// ---- host launchers ------------------------------------------------------------------------------

hipError_t launch_extract(const Launch<ExtractJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    ks_launch(extract_kernel, dim3((unsigned)L.total_blocks), dim3(EXTRACT_TPB), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_anchor(const Launch<AnchorJob> &L, int w_in, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    dim3 g((unsigned)L.total_blocks), b(ANCHOR_TPB);
    switch (w_in) {
        case 1: ks_launch(anchor_kernel<1>, g, b, 0, s, L); break;
        case 2: ks_launch(anchor_kernel<2>, g, b, 0, s, L); break;
        case 3: ks_launch(anchor_kernel<3>, g, b, 0, s, L); break;
        case 4: ks_launch(anchor_kernel<4>, g, b, 0, s, L); break;
        case 5: ks_launch(anchor_kernel<5>, g, b, 0, s, L); break;
        case 6: ks_launch(anchor_kernel<6>, g, b, 0, s, L); break;
        case 7: ks_launch(anchor_kernel<7>, g, b, 0, s, L); break;
        case 8: ks_launch(anchor_kernel<8>, g, b, 0, s, L); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finish(const Launch<ChainJob> &L, int nw, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    dim3 g((unsigned)L.total_blocks), b(FINISH_TPB);
    switch (nw) {
        case 0: ks_launch(finish_any_kernel, g, b, 0, s, L); break;
        case 1: ks_launch(finish_kernel<1>, g, b, 0, s, L); break;
        case 2: ks_launch(finish_kernel<2>, g, b, 0, s, L); break;
        case 3: ks_launch(finish_kernel<3>, g, b, 0, s, L); break;
        case 4: ks_launch(finish_kernel<4>, g, b, 0, s, L); break;
        case 5: ks_launch(finish_kernel<5>, g, b, 0, s, L); break;
        case 6: ks_launch(finish_kernel<6>, g, b, 0, s, L); break;
        case 7: ks_launch(finish_kernel<7>, g, b, 0, s, L); break;
        case 8: ks_launch(finish_kernel<8>, g, b, 0, s, L); break;
        case 9: ks_launch(finish_kernel<9>, g, b, 0, s, L); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_chain(const Launch<ChainJob> &L, int nw, bool lanes, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    dim3 b(CHAIN_TPB);
    if (lanes) {
        dim3 g((unsigned)((L.total_blocks + CHAIN_TPB - 1) / CHAIN_TPB));
        switch (nw) {
            case 0: ks_launch(chain_lanes_kernel<0>, g, b, 0, s, L); break;
            case 1: ks_launch(chain_lanes_kernel<1>, g, b, 0, s, L); break;
            case 2: ks_launch(chain_lanes_kernel<2>, g, b, 0, s, L); break;
            case 3: ks_launch(chain_lanes_kernel<3>, g, b, 0, s, L); break;
            case 4: ks_launch(chain_lanes_kernel<4>, g, b, 0, s, L); break;
            case 5: ks_launch(chain_lanes_kernel<5>, g, b, 0, s, L); break;
            case 6: ks_launch(chain_lanes_kernel<6>, g, b, 0, s, L); break;
            case 7: ks_launch(chain_lanes_kernel<7>, g, b, 0, s, L); break;
            case 8: ks_launch(chain_lanes_kernel<8>, g, b, 0, s, L); break;
            case 9: ks_launch(chain_lanes_kernel<9>, g, b, 0, s, L); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    dim3 g((unsigned)L.total_blocks);
    switch (nw) {
        case 1: ks_launch(chain_kernel<1>, g, b, 0, s, L); break;
        case 2: ks_launch(chain_kernel<2>, g, b, 0, s, L); break;
        case 3: ks_launch(chain_kernel<3>, g, b, 0, s, L); break;
        case 4: ks_launch(chain_kernel<4>, g, b, 0, s, L); break;
        case 5: ks_launch(chain_kernel<5>, g, b, 0, s, L); break;
        case 6: ks_launch(chain_kernel<6>, g, b, 0, s, L); break;
        case 7: ks_launch(chain_kernel<7>, g, b, 0, s, L); break;
        case 8: ks_launch(chain_kernel<8>, g, b, 0, s, L); break;
        case 9: ks_launch(chain_kernel<9>, g, b, 0, s, L); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ks
