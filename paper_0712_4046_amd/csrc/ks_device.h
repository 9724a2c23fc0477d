// ks_device.h -- device-side building blocks shared by the libksmul kernels (gfx950, wave64).
//
// The one primitive every stage leans on is exact carry resolution of a multi-limb integer
// given as signed 64-bit "limb columns":  V = sum_j v_j 2^(32 j).  Packing (the overlapping
// sums of Section 3.4 and the signed evaluations of Section 3.3), recombining products and
// exact halving (Sections 3.3, 3.4) all reduce to it.  Two local steps bring every position
// to a value u_j in [-1, 2^32]; what remains is a carry k in {-1, 0, +1} that may travel
// arbitrarily far.  The carry out of position j is a monotone map of the carry into it,
// determined by u_j alone, so the maps compose associatively and one parallel scan over
// them resolves every carry:
//   within a thread   -- sequential composition of its items;
//   within a wave     -- shuffle scan (6 steps on 64 lanes);
//   within a block    -- wave aggregates in LDS;
//   across blocks     -- single-pass decoupled look-back on epoch-tagged status words,
//                        a job's blocks ordered by tickets from the job's own counter so a
//                        block only ever waits on blocks that are already running.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ks_jobs.h"

namespace ks {

// ---- carry maps ------------------------------------------------------------------------------
// A map {-1,0,1} -> {-1,0,1} packed as three 2-bit fields: field x (x = k+1) holds out(k)+1.
typedef uint32_t cmap;
constexpr cmap CMAP_ID = 0u | (1u << 2) | (2u << 4);

__device__ __forceinline__ int cmap_apply(cmap m, int k) { return (int)((m >> (2 * (k + 1))) & 3u) - 1; }

// first f, then g
__device__ __forceinline__ cmap cmap_then(cmap f, cmap g) {
    cmap r = 0;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        uint32_t fx = (f >> (2 * x)) & 3u;
        r |= ((g >> (2 * fx)) & 3u) << (2 * x);
    }
    return r;
}

// carry-out map of a position whose pre-carry value is u in [-1, 2^32]
__device__ __forceinline__ cmap cmap_of(int64_t u) {
    if (u == -1) return 0u | (0u << 2) | (1u << 4);                   // -1,-1, 0
    if (u == 0) return 0u | (1u << 2) | (1u << 4);                    // -1, 0, 0
    if (u == (int64_t)0xffffffffLL) return 1u | (1u << 2) | (2u << 4); //  0, 0, 1
    if (u == (int64_t)0x100000000LL) return 1u | (2u << 2) | (2u << 4); //  0, 1, 1
    return 1u | (1u << 2) | (1u << 4);                                //  0, 0, 0
}

// ---- local steps: v_j (int64 column) -> u_j in [-1, 2^32] -----------------------------------
// u_j depends on v_j, v_{j-1}, v_{j-2}:
//   t_j = lo32(v_j) + (v_{j-1} >> 32)          in [-2^31, 2^32 + 2^31)
//   u_j = lo32(t_j) + (t_{j-1} >> 32)           in [-1, 2^32]
__device__ __forceinline__ int64_t t_of(int64_t v, int64_t vprev) {
    return (int64_t)(uint32_t)(uint64_t)v + (vprev >> 32);
}
__device__ __forceinline__ int64_t u_of(int64_t v, int64_t v1, int64_t v2) {
    int64_t t = t_of(v, v1), tp = t_of(v1, v2);
    return (int64_t)(uint32_t)(uint64_t)t + (tp >> 32);
}

// ---- status words for the look-back -----------------------------------------------------------
// bits 63..32 epoch of the launch, bits 9..8 flag (1 aggregate map, 2 inclusive carry),
// bits 7..0 payload (map, or carry + 1).  The whole message travels inside one 64-bit word,
// so relaxed device-scope atomics suffice: no other memory is published through it, and the
// limbs a block writes are only read by later kernels on the stream.
constexpr uint32_t LB_AGG = 1, LB_INC = 2;
constexpr uint64_t LB_SPIN_LIMIT = 1ull << 22;

__device__ __forceinline__ void lb_publish(uint64_t *st, uint32_t epoch, uint32_t flag, uint32_t payload) {
    uint64_t w = ((uint64_t)epoch << 32) | ((uint64_t)flag << 8) | payload;
    __hip_atomic_store(st, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_load(const uint64_t *st) {
    return __hip_atomic_load(const_cast<uint64_t *>(st), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block ticket of a carry-scan job of several blocks: the job's blocks draw their positions in
// the look-back order from the job's own counter, so a block only ever waits on blocks that
// are already running; the block that draws the last ticket puts the counter back to zero for
// the next launch (launches of one stream run one after the other).  Jobs of one block need
// no ticket.  No two jobs share a counter, and a batch's launch interleaves its jobs' blocks,
// so that the atomics of the blocks running at one time spread over many words.
__device__ __forceinline__ int64_t job_ticket(uint64_t *ctr, int64_t nblocks) {
    const uint64_t t = __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int64_t)t == nblocks - 1) __hip_atomic_store(ctr, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (int64_t)t;
}

__device__ __forceinline__ void set_status(uint32_t *devstat, uint32_t bit) {
    __hip_atomic_fetch_or(devstat, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Resolve the carry into block `blk` of a chain whose status words start at `st`.  Called by
// all 64 lanes of one wave (the same `agg`, this block's aggregate map, on every lane); every
// lane returns the carry in.  Lane l watches block p - l of a window of 64 predecessors, so
// one round of loads covers 64 blocks: if some block of the window has published its
// inclusive carry, the maps of the blocks after it are composed by a shuffle reduction and
// applied to it; if every block of the window has published at least its aggregate map, the
// window's composition is kept and the window moves 64 blocks down; otherwise the wave waits.
__device__ __forceinline__ int lb_resolve(uint64_t *st, int64_t blk, uint32_t epoch, cmap agg, uint32_t *devstat) {
    const int lane = threadIdx.x & 63;
    if (blk == 0) {
        if (lane == 0) lb_publish(st, epoch, LB_INC, (uint32_t)(cmap_apply(agg, 0) + 1));
        return 0;
    }
    if (lane == 0) lb_publish(st + blk, epoch, LB_AGG, agg);
    cmap acc = CMAP_ID;  // composition of the blocks above the window, up to blk - 1
    int64_t top = blk - 1;
    uint64_t spins = 0;
    int carry = 0;
    for (;;) {
        const int64_t p = top - lane;
        const bool in = p >= 0;
        const uint64_t w = in ? lb_load(st + p) : 0ull;
        const bool fresh = in && (uint32_t)(w >> 32) == epoch;
        const uint32_t flag = fresh ? (uint32_t)(w >> 8) & 3u : 0u;
        const uint64_t inc = __ballot(in && flag == LB_INC);
        const uint64_t wait = __ballot(in && flag == 0);
        // lanes below the nearest inclusive block (or the whole window) must have a map
        const int first_inc = inc ? __builtin_ctzll(inc) : 64;
        const uint64_t need = first_inc == 64 ? ~0ull : ((1ull << first_inc) - 1ull);
        if (wait & need) {
            if (++spins > LB_SPIN_LIMIT) {  // never expected; keeps every wave finite
                if (lane == 0) set_status(devstat, KS_DEVSTAT_LOOKBACK);
                carry = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        // compose the maps of lanes first_inc-1 .. 0 (blocks in increasing order)
        cmap m = (lane < first_inc && in) ? (cmap)(w & 0xffu) : CMAP_ID;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const cmap o = (cmap)__shfl_down((int)m, dd, 64);
            if ((lane & (2 * dd - 1)) == 0) m = cmap_then(lane + dd < 64 ? o : CMAP_ID, m);
        }
        m = (cmap)__shfl((int)m, 0, 64);
        acc = cmap_then(m, acc);
        if (first_inc < 64) {
            const int c = (int)((uint32_t)__shfl((int)(uint32_t)(w & 0xffu), first_inc, 64)) - 1;
            carry = cmap_apply(acc, c);
            break;
        }
        top -= 64;
        if (top < 0) {  // every block down to block 0 composed: block 0's carry in is 0
            carry = cmap_apply(acc, 0);
            break;
        }
    }
    if (lane == 0) lb_publish(st + blk, epoch, LB_INC, (uint32_t)(cmap_apply(agg, carry) + 1));
    return carry;
}

// ---- block-wide carry scan ---------------------------------------------------------------------
// Each of the TPB threads holds IPT consecutive pre-carry values u[]; on return out[] holds the
// normalised limbs and the function returns the carry out of the thread's last item.
// `st` points at the status words of this chain, `blk` is the block's index in the chain.
template <int TPB, int IPT>
struct BlockCarryScan {
    struct Smem {
        cmap wave_agg[TPB / 64];
        int carry_in;
    };

    __device__ static int run(Smem &sm, const int64_t (&u)[IPT], uint32_t (&out)[IPT], uint64_t *st, int64_t blk,
                              uint32_t epoch, uint32_t *devstat) {
        const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
        cmap maps[IPT];
        cmap mine = CMAP_ID;
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            maps[q] = cmap_of(u[q]);
            mine = cmap_then(mine, maps[q]);
        }
        // inclusive scan over the wave
        cmap inc = mine;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            cmap o = (cmap)__shfl_up((int)inc, d, 64);
            if (lane >= d) inc = cmap_then(o, inc);
        }
        cmap excl = (cmap)__shfl_up((int)inc, 1, 64);
        if (lane == 0) excl = CMAP_ID;
        if (lane == 63) sm.wave_agg[wv] = inc;
        __syncthreads();
        if (wv == 0) {
            cmap agg = CMAP_ID;
#pragma unroll
            for (int w = 0; w < TPB / 64; ++w) agg = cmap_then(agg, sm.wave_agg[w]);
            // a job of one block has no predecessors and no successors: nothing to publish
            const int c = st ? lb_resolve(st, blk, epoch, agg, devstat) : 0;
            if (lane == 0) sm.carry_in = c;
        }
        __syncthreads();
        cmap before = CMAP_ID;
        for (int w = 0; w < wv; ++w) before = cmap_then(before, sm.wave_agg[w]);
        before = cmap_then(before, excl);
        int k = cmap_apply(before, sm.carry_in);
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            out[q] = (uint32_t)(uint64_t)(u[q] + k);
            k = cmap_apply(maps[q], k);
        }
        return k;
    }
};

// lo:hi (96 bits) += a * b: v_mad_u64_u32 accumulates the 32x32-bit product into 64 bits and
// hands its carry to a v_addc into the top 32 bits
__device__ __forceinline__ void mac96(uint64_t &lo, uint32_t &hi, uint32_t a, uint32_t b) {
    uint64_t cc;
    asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
        "v_addc_co_u32_e64 %2, %1, 0, %2, %1"
        : "+v"(lo), "=&s"(cc), "+v"(hi)
        : "v"(a), "v"(b));
}

// ---- loads through global (not flat) pointers ---------------------------------------------------
// A flat load also counts against the LDS wait counter, so a kernel that prefetches from
// global memory while it works out of LDS would drain its prefetches at every LDS wait.
template <class T>
__device__ __forceinline__ T ldg(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}

// N consecutive words through the widest global vector loads (dword alignment is enough):
// a wave-wide load instruction costs the address unit one pass per cache line it touches, so
// four words in one instruction instead of four cost a quarter
typedef uint32_t u32x2 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3), aligned(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4), aligned(4)));

template <int N>
__device__ __forceinline__ void ldg_words(const uint32_t *p, uint32_t *o) {
    int t = 0;
#pragma unroll
    for (; t + 4 <= N; t += 4) {
        const u32x4 v = *(const __attribute__((address_space(1))) u32x4 *)(p + t);
        o[t] = v.x;
        o[t + 1] = v.y;
        o[t + 2] = v.z;
        o[t + 3] = v.w;
    }
    if constexpr (N % 4 == 3) {
        const u32x3 v = *(const __attribute__((address_space(1))) u32x3 *)(p + t);
        o[t] = v.x;
        o[t + 1] = v.y;
        o[t + 2] = v.z;
    } else if constexpr (N % 4 == 2) {
        const u32x2 v = *(const __attribute__((address_space(1))) u32x2 *)(p + t);
        o[t] = v.x;
        o[t + 1] = v.y;
    } else if constexpr (N % 4 == 1) {
        o[t] = *(const __attribute__((address_space(1))) uint32_t *)(p + t);
    }
}

// N consecutive words stored through the widest global vector stores (dword alignment)
template <int N>
__device__ __forceinline__ void stg_words(uint32_t *p, const uint32_t *v) {
    int t = 0;
#pragma unroll
    for (; t + 4 <= N; t += 4) {
        u32x4 x;
        x.x = v[t];
        x.y = v[t + 1];
        x.z = v[t + 2];
        x.w = v[t + 3];
        *(__attribute__((address_space(1))) u32x4 *)(p + t) = x;
    }
    if constexpr (N % 4 == 3) {
        u32x3 x;
        x.x = v[t];
        x.y = v[t + 1];
        x.z = v[t + 2];
        *(__attribute__((address_space(1))) u32x3 *)(p + t) = x;
    } else if constexpr (N % 4 == 2) {
        u32x2 x;
        x.x = v[t];
        x.y = v[t + 1];
        *(__attribute__((address_space(1))) u32x2 *)(p + t) = x;
    } else if constexpr (N % 4 == 1) {
        *(__attribute__((address_space(1))) uint32_t *)(p + t) = v[t];
    }
}

template <class T>
__device__ __forceinline__ void stg(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

// The scalar fields of a launch that block bodies need, passed by value: a block body that took
// the whole launch by reference (or by value) lost the kernel arguments' scalar loads.
struct LaunchCtl {
    uint64_t *status;
    uint64_t *ctrs;
    uint32_t *devstat;
    uint32_t epoch;
};
template <class J>
__device__ __forceinline__ LaunchCtl ctl_of(const Launch<J> &L) {
    return LaunchCtl{L.status, L.ctrs, L.devstat, L.epoch};
}

// ---- XCD-aware block order ----------------------------------------------------------------------
// The dispatcher deals the blocks of a launch to the GPU's 8 XCDs in turn (block b to XCD
// b mod 8), and each XCD has an L2 of its own.  Blocks that re-read the same data (the anchors
// of one product, the matrix-core blocks of one product) share that L2 only if they run on one
// XCD, so block b of n takes the logical index (b mod 8) floor(n/8) + floor(b/8): the logical
// blocks [x floor(n/8), (x+1) floor(n/8)) all run on one XCD.  The last n mod 8 blocks keep their
// index.  A bijection of [0, n), so every logical block runs exactly once.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
    const int64_t per = n / NUM_XCD;
    if (b >= per * NUM_XCD) return b;
    return (b % NUM_XCD) * per + b / NUM_XCD;
}

// ---- job lookup: block index -> (job, block within job) ----------------------------------------
// Inline jobs: all block0 values are loaded at once (independent scalar loads, one round
// trip).  Device tables: one load from the block -> job map.
template <class J>
__device__ __forceinline__ J find_job(const Launch<J> &L, int64_t blk, int64_t &local) {
    if (L.table == nullptr) {
        int j = 0;
#pragma unroll
        for (int q = 1; q < MAX_INLINE_JOBS; ++q) {
            const int64_t b0 = L.jobs[q].block0;
            if (q < L.njobs && blk >= b0) j = q;
        }
        local = blk - L.jobs[j].block0;
        return L.jobs[j];
    }
    const J job = L.table[L.block_job[blk]];
    local = blk - job.block0;
    return job;
}

template <class T>
__device__ __forceinline__ T *at(uintptr_t base, T *rel) {
    return reinterpret_cast<T *>(base + reinterpret_cast<uintptr_t>(rel));
}

// turn a job's relative pointers into addresses
template <class J> __device__ __forceinline__ void rebase(J &, const Launch<J> &);
template <> __device__ __forceinline__ void rebase(PackJob &J, const Launch<PackJob> &L) {
    J.coeffs = at(L.base_in, J.coeffs);
    J.out = at(L.base_ws, J.out);
}
template <> __device__ __forceinline__ void rebase(MulJob &J, const Launch<MulJob> &L) {
    J.a = at(L.base_ws, J.a);
    J.b = at(L.base_ws, J.b);
    J.cols = at(L.base_ws, J.cols);
}
template <> __device__ __forceinline__ void rebase(NormJob &J, const Launch<NormJob> &L) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        J.term[q].cols = at(L.base_ws, J.term[q].cols);
        J.term[q].a = at(L.base_ws, J.term[q].a);
        J.term[q].b = at(L.base_ws, J.term[q].b);
    }
    J.out = at(L.base_ws, J.out);
    J.out2 = at(L.base_ws, J.out2);
}
template <> __device__ __forceinline__ void rebase(ExtractJob &J, const Launch<ExtractJob> &L) {
    J.src = at(L.base_ws, J.src);
    J.out = at(L.base_out, J.out);
}
template <> __device__ __forceinline__ void rebase(AnchorJob &J, const Launch<AnchorJob> &L) {
    J.f = at(L.base_in, J.f);
    J.g = at(L.base_in, J.g);
    J.anchors = at(L.base_ws, J.anchors);
    J.anchors2 = at(L.base_ws, J.anchors2);
}
template <> __device__ __forceinline__ void rebase(ChainJob &J, const Launch<ChainJob> &L) {
    J.A = at(L.base_ws, J.A);
    J.B = at(L.base_ws, J.B);
    J.anchors = at(L.base_ws, J.anchors);
    J.hbuf = at(L.base_ws, J.hbuf);
    J.out = at(L.base_out, J.out);
}

template <> __device__ __forceinline__ void rebase(DigitJob &J, const Launch<DigitJob> &L) {
    J.limbs = at(L.base_ws, J.limbs);
    J.out = at(L.base_ws, J.out);
    J.zero = at(L.base_ws, J.zero);
}
template <> __device__ __forceinline__ void rebase(MfmaJob &J, const Launch<MfmaJob> &L) {
    J.ad = at(L.base_ws, J.ad);
    J.bd = at(L.base_ws, J.bd);
    J.cols = at(L.base_ws, J.cols);
}

template <> __device__ __forceinline__ void rebase(NttJob &J, const Launch<NttJob> &L) {
    J.a = at(L.base_ws, J.a);
    J.x = at(L.base_ws, J.x);
    J.y = at(L.base_ws, J.y);
}

template <class J>
__device__ __forceinline__ J get_job(const Launch<J> &L, int64_t blk, int64_t &local) {
    J job = find_job(L, blk, local);
    rebase(job, L);
    return job;
}

// ---- arithmetic modulo the transform engine's primes --------------------------------------------

struct NttPrime {
    uint32_t p;
    uint32_t pn;  // -p^-1 mod 2^32
};

__host__ __device__ constexpr uint32_t neg_inv32(uint32_t p) {
    uint32_t x = p;  // Newton's iteration for p^-1 mod 2^32 (p odd): 5 steps from 3 bits
    for (int i = 0; i < 5; ++i) x *= 2u - p * x;
    return 0u - x;
}

// a^-1 mod p (extended Euclid), for the constant of the Chinese remainder step
constexpr uint64_t inv_mod(uint64_t a, uint64_t p) {
    int64_t t = 0, nt = 1, r = (int64_t)p, nr = (int64_t)(a % p);
    while (nr != 0) {
        const int64_t qq = r / nr;
        const int64_t t2 = t - qq * nt, r2 = r - qq * nr;
        t = nt;
        nt = t2;
        r = nr;
        nr = r2;
    }
    return (uint64_t)(t < 0 ? t + (int64_t)p : t);
}
// P0^-1 R mod P1 (Montgomery form, R = 2^32): multiplying by it divides by P0 mod P1
constexpr uint32_t NTT_CRT_C = (uint32_t)(inv_mod(NTT_P0, NTT_P1) * (((uint64_t)1 << 32) % NTT_P1) % NTT_P1);
static_assert(inv_mod(NTT_P0, NTT_P1) * (NTT_P0 % NTT_P1) % NTT_P1 == 1, "P0 inverse mod P1");

__host__ __device__ constexpr NttPrime ntt_prime_c(int q) {
    return q == 0 ? NttPrime{NTT_P0, neg_inv32(NTT_P0)} : NttPrime{NTT_P1, neg_inv32(NTT_P1)};
}
__device__ __forceinline__ NttPrime ntt_prime(int q) { return ntt_prime_c(q); }

// Residues may be held partly reduced, below 2p or 4p: with p < 2^30, 4p still fits in a
// 32-bit word.  s < 2p -> [0, p) and s < 4p -> [0, 2p), each as min(s, s - c): the subtraction
// wraps to a large value exactly when s < c.
__device__ __forceinline__ uint32_t red1(uint32_t s, uint32_t p) { return min(s, s - p); }
__device__ __forceinline__ uint32_t red2(uint32_t s, uint32_t p) { return min(s, s - 2u * p); }

// a b R^-1 mod p below 2p (Montgomery reduction without its final subtraction) whenever
// a b < p 2^32 -- any 32-bit a with b < p, or a, b < 2p, or a < 4p with b < p, as 4p < 2^32:
// t = a b, m = t p' mod 2^32, and (t + m p) / 2^32 < a b / 2^32 + p < 2p, with t + m p < 2^63
// not wrapping.  The compiler turns it into three multiply-adds (v_mad_u64_u32, v_mul_lo_u32,
// v_mad_u64_u32).
__device__ __forceinline__ uint32_t mmul_lazy(uint32_t a, uint32_t b, NttPrime P) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * P.pn;
    return (uint32_t)((t + (uint64_t)m * P.p) >> 32);
}
// the same, fully reduced (below p)
__device__ __forceinline__ uint32_t mmul(uint32_t a, uint32_t b, NttPrime P) { return red1(mmul_lazy(a, b, P), P.p); }
__device__ __forceinline__ uint32_t madd(uint32_t a, uint32_t b, uint32_t p) {
    const uint32_t s = a + b;
    return s >= p ? s - p : s;
}
__device__ __forceinline__ uint32_t msub(uint32_t a, uint32_t b, uint32_t p) { return a >= b ? a - b : a + p - b; }

// the value below P0 P1 with residues x0 mod P0 and x1 mod P1 (Chinese remainder theorem):
// x0 + P0 ((x1 - x0) P0^-1 mod P1)
__device__ __forceinline__ uint64_t crt2(uint32_t x0, uint32_t x1) {
    const uint32_t x0m = x0 >= NTT_P1 ? x0 - NTT_P1 : x0;  // x0 < P0 < 2 P1
    const uint32_t t = mmul(msub(x1, x0m, NTT_P1), NTT_CRT_C, NttPrime{NTT_P1, neg_inv32(NTT_P1)});
    return (uint64_t)x0 + (uint64_t)NTT_P0 * t;
}

// ---- small helpers ------------------------------------------------------------------------------

// bits [s, s+32) of the w-limb integer c (two's complement when sgn; bits below 0 read 0)
__device__ __forceinline__ uint32_t coeff_word(const uint32_t *c, int w, bool sgn, int64_t s) {
    uint32_t fill = (sgn && (c[w - 1] >> 31)) ? 0xffffffffu : 0u;
    if (s < 0) {
        int r = (int)(-s);
        uint32_t lo = c[0];
        return r >= 32 ? 0u : (lo << r);
    }
    int64_t q = s >> 5;
    int o = (int)(s & 31);
    uint32_t a = q < w ? c[q] : fill;
    if (o == 0) return a;
    uint32_t b = q + 1 < w ? c[q + 1] : fill;
    return (a >> o) | (b << (32 - o));
}

// bits [s, s+32) of an n-limb non-negative integer (limbs at or above n read 0)
__device__ __forceinline__ uint32_t bits_word(const uint32_t *x, int64_t n, int64_t s) {
    int64_t q = s >> 5;
    int o = (int)(s & 31);
    uint32_t a = (q >= 0 && q < n) ? x[q] : 0u;
    if (o == 0) return a;
    uint32_t b = (q + 1 >= 0 && q + 1 < n) ? x[q + 1] : 0u;
    return (a >> o) | (b << (32 - o));
}

// floor(a / d) for 0 <= a < 2^40 with recip = div_recip(d) computed on the host
__device__ __forceinline__ int64_t div_by(int64_t a, uint64_t recip) {
    return recip == 0 ? a : (int64_t)__umul64hi((uint64_t)a, recip);
}

}  // namespace ks
