// ks_mul_mfma.hip -- integer products on the int8 matrix cores (v_mfma_i32_32x32x32_i8).
//
// An integer product is a convolution of digit sequences: with balanced 8-bit digits a_i, b_j
// (values -128..127, exactly the signed int8 operands: A = sum_i a_i 256^i, see
// digitize_kernel), C[k] = sum_i a_i b_{k-i} and A*B = sum_k C[k] 2^(8k).  Writing k = 32 r + s
// (output row r: a 32-digit block) and splitting the shift into 32-digit blocks t,
//     C[32 r + s] = sum_t sum_{q<32} b[32 t + s - q] * a[32 (r - t) + q],
// each block shift t is a 32x32x32 matrix product: matrix rows s (the digit within an output
// row), matrix columns r, contraction q; the left matrix is a Toeplitz tile of b and the right
// one holds contiguous 32-digit runs of a.  One v_mfma_i32_32x32x32_i8 computes it,
// accumulating exactly in int32 (at most 32 * 128^2 in absolute value per step; a wave takes at
// most 4064 steps).  Against 7-bit digits (0..127) the balanced digits need 8/7 fewer per
// operand, (8/7)^2 = 1.31x fewer multiply-adds per product.
//
// Lane layout of v_mfma_i32_32x32x32_i8 (checked on the device): lane l supplies row (left
// operand) or column (right operand) l % 32 and contraction indices 16 (l / 32) .. + 15 as 16
// bytes; result register i of lane l is matrix row 8 (i / 4) + 4 (l / 32) + (i % 4), column
// l % 32.  So a lane's registers 4 a .. 4 a + 3 hold the four digits of one limb: limb
// 2 a + l / 32 of output row r = l % 32 of the tile, assembled in the lane itself.
//
// A block covers MFMA_RT tiles (32 output rows each: 32 * 32 * MFMA_RT output digits =
// MFMA_LIMBS limbs), one part of the range of t and one of `rgroups` groups of the residues of
// t mod 32.  Wave w takes the shifts of its part congruent to w mod MFMA_WAVES that fall in
// the block's residue group: MFMA_CLASSES / rgroups residue classes, one after the other (one
// class when rgroups = 4: a single long chain of steps, whose start-up latency is paid once).
// Within a class t advances by 32, which moves every tile's a-runs by exactly one tile: the
// a-fragment of tile rt at one step is that of tile rt-1 at the step before.  So a step loads
// one new a-fragment (16 contiguous bytes per lane) and one Toeplitz b-window (68 bytes, one
// dword per lane, spread by lane shuffles and realigned with v_alignbyte) straight from global
// memory, PF steps ahead, and issues MFMA_RT matrix operations.  At the end every wave turns
// its digit sums into limb values in registers and stores them into an LDS slice of its own;
// the block adds the waves' slices and adds its limb columns into the product's column buffer
// with 64-bit atomics, so any number of blocks may share a row group (the only block of a row
// group stores its columns instead, into a buffer nobody clears).
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---- digits ------------------------------------------------------------------------------------

// Balanced base-256 digits.  With bytes b_k of the limb array (4 n of them) and carries
// c_0 = 0, c_{k+1} = [b_k + c_k >= 128], digit d_k = b_k + c_k - 256 c_{k+1} lies in [-128, 127]
// and sum_k d_k 256^k = sum_k b_k 256^k, with the top digit d_{4n} = c_{4n}.  A byte 0x7f passes
// its carry on and any other byte decides it, so the carry into limb q comes from the nearest
// lower limb that is not 0x7f7f7f7f (zero below limb 0): from a lane of the same wave (ballot),
// else from a backward search of the limbs below the wave, 64 per round by the whole wave.
//
// out[x] for x in [0, len): digit (reversed ? base - x : x - base), 0 outside [0, 4n]; then
// zero[0, zero_len).  Four bytes (one limb's digits) per thread; the four digits of a thread
// start at a multiple of 4 (base is 3 mod 4 when reversed, 0 mod 4 otherwise).
__device__ __forceinline__ bool carry_out_of(uint32_t w) {  // limb not 0x7f7f7f7f: its carry out
    bool c = false;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const uint32_t b = (w >> (8 * t)) & 0xffu;
        c = b >= 128u || (b == 127u && c);
    }
    return c;
}

__global__ __launch_bounds__(256) void digitize_kernel(Launch<DigitJob> L) {
    int64_t local;
    const DigitJob J = get_job(L, (int64_t)blockIdx.x, local);
    const int lane = threadIdx.x & 63;
    const int64_t x0 = (local * 256 + threadIdx.x) * 4;
    const bool rev = J.reversed != 0;
    // the limb whose four digits this thread's position holds (lanes take consecutive limbs,
    // ascending with the lane, or descending when reversed -- also past len, where nothing is
    // written, so that every lane of a wave stands for its limb in the carry search)
    const int64_t dlow = rev ? J.base - x0 - 3 : x0 - J.base;  // lowest digit, a multiple of 4
    const int64_t q = dlow >> 2;
    const bool real = q >= 0 && q < J.n;
    const uint32_t w = real ? ldg(J.limbs + q) : 0u;
    const bool decides = q < 0 || (real && w != 0x7f7f7f7fu);  // below limb 0: carry 0
    const bool cout = real && carry_out_of(w);
    const uint64_t dec = __ballot(decides), gen = __ballot(decides && cout);
    // lanes holding lower limbs than this lane's
    const uint64_t lower = rev ? (lane == 63 ? 0ull : (~0ull << (lane + 1))) : ((1ull << lane) - 1ull);
    // carry into the wave's lowest limb: searched below it when some lane needs it
    const int64_t qmin = rev ? q - (63 - lane) : q - lane;  // lane 63 (reversed) or lane 0 holds it
    const int64_t wq = __shfl(qmin, 0, 64);
    bool wave_cin = false;
    if (__ballot((dec & lower) == 0ull && q >= 0 && q <= J.n) != 0ull) {
        for (int64_t top = wq - 1; top >= 0; top -= 64) {
            const int64_t qq = top - lane;  // lane 0 holds the highest limb of the round
            const bool okq = qq >= 0 && qq < J.n;
            const uint32_t ww = okq ? ldg(J.limbs + qq) : 0u;
            const bool d2 = qq < 0 || (okq && ww != 0x7f7f7f7fu);
            const uint64_t dm = __ballot(d2);
            if (dm) {
                const int src = __builtin_ctzll(dm);  // the nearest deciding limb
                wave_cin = ((__ballot(d2 && okq && carry_out_of(ww)) >> src) & 1ull) != 0ull;
                break;
            }
        }
    }
    const uint64_t cand = dec & lower;
    bool c;
    if (cand) {
        const int src = rev ? __builtin_ctzll(cand) : 63 - __builtin_clzll(cand);
        c = ((gen >> src) & 1ull) != 0ull;
    } else {
        c = wave_cin;
    }
    uint32_t d[4] = {0u, 0u, 0u, 0u};
    if (real) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t s = ((w >> (8 * t)) & 0xffu) + (c ? 1u : 0u);
            c = s >= 128u;
            d[t] = (s - (c ? 256u : 0u)) & 0xffu;
        }
    } else if (q == J.n) {
        d[0] = c ? 1u : 0u;  // the top carry
    }
    if (x0 < J.len) {
        const uint32_t word = rev ? (d[3] | (d[2] << 8) | (d[1] << 16) | (d[0] << 24))
                                  : (d[0] | (d[1] << 8) | (d[2] << 16) | (d[3] << 24));
        *reinterpret_cast<uint32_t *>(J.out + x0) = word;
    } else if (x0 - J.len < J.zero_len) {
        *reinterpret_cast<uint32_t *>(J.zero + (x0 - J.len)) = 0u;
    }
}

// ---- products ----------------------------------------------------------------------------------

__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// loads through global (not flat) pointers, so waiting for LDS traffic never waits for them
typedef __attribute__((address_space(1))) const v4i gv4i;
typedef __attribute__((address_space(1))) const uint32_t gu32;

__device__ __forceinline__ v4i mfma_frag(const uint8_t *arow, int64_t R) {
    return *(gv4i *)(arow + 32 * R);
}

// b-operand of one shift from its window: lane l holds dword l (l <= 16) of the 68 bytes the
// shift reads; lane (m, g) needs dwords sel .. sel+4 and the 16 bytes at byte offset sh in them
__device__ __forceinline__ v4i mfma_bop(uint32_t win, int sel, uint32_t sh) {
    uint32_t w[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) w[i] = (uint32_t)__shfl((int)win, sel + i, 64);
    v4i b;
    b[0] = (int)__builtin_amdgcn_alignbyte(w[1], w[0], sh);
    b[1] = (int)__builtin_amdgcn_alignbyte(w[2], w[1], sh);
    b[2] = (int)__builtin_amdgcn_alignbyte(w[3], w[2], sh);
    b[3] = (int)__builtin_amdgcn_alignbyte(w[4], w[3], sh);
    return b;
}

template <int RT>
__global__ __launch_bounds__(MFMA_TPB) void mul_mfma_kernel(Launch<MfmaJob> L) {
    constexpr int MFMA_ROWS = mfma_rows(RT), MFMA_LIMBS = mfma_limbs(RT);
    constexpr int PF = 8;  // steps loaded ahead (the b-window is consumed one step early)
    constexpr int UN = RT > PF ? RT : PF;  // steps per unrolled group: slot and ring indices are constants
    static_assert(UN % RT == 0 && UN % PF == 0, "fragment slots and prefetch ring must divide the unroll");
    // limb sums of each wave: limb w of output row rb (w < 8, rb < MFMA_ROWS) at
    // w * MFMA_ROWS + (rb ^ 8 w), so that both the waves' stores and the block's sums meet few
    // LDS bank conflicts
    __shared__ long long D[MFMA_WAVES][MFMA_LIMBS];

    int64_t local;
    // the blocks of one product share its digit buffers: keep them on one XCD's L2
    const MfmaJob J = get_job(L, xcd_block((int64_t)blockIdx.x, L.total_blocks), local);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 31, g = lane >> 5;
    // block index within the job: (row group, part, residue group), the residue group fastest
    const int64_t per_grp = J.splits * J.rgroups;
    const int64_t grp = local / per_grp, rem = local - grp * per_grp;
    const int64_t part = rem / J.rgroups;
    const int rg = (int)(rem - part * J.rgroups);
    const int cpw = MFMA_CLASSES / (int)J.rgroups;  // residue classes per wave
    const int64_t S0 = grp * MFMA_ROWS;  // first output row (32-digit block) of the block

    // shifts t with a[32 (s - t) ..] and b[32 t ..] both inside the operands for some row s
    // of the block, cut into parts
    int64_t tlo = S0 - J.nA32 + 1;
    if (tlo < 0) tlo = 0;
    int64_t thi = S0 + MFMA_ROWS - 1;
    if (thi > J.nB32 - 1) thi = J.nB32 - 1;
    const int64_t ta = tlo + part * J.part;
    int64_t tb = ta + J.part;
    if (tb > thi + 1) tb = thi + 1;

    v16i acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[rt][i] = 0;

    // lane (m, g) supplies a-row m and b-column m, contraction bytes 16 g .. 16 g + 15:
    //   a-fragment of the tile whose rows start at R: ad[a_front + 32 (R + m) + 16 g ..]
    //   b-bytes of shift t: bd[b_top - 32 t - m + 16 g ..]; the wave loads the dword-aligned
    //   window from bd[wb - 32 t] (one dword per lane) and lanes gather theirs by shuffles
    const uint8_t *arow = J.ad + J.a_front + 32 * m + 16 * g;
    const uint32_t sh = (uint32_t)((J.b_top - m) & 3);
    const int64_t wb = (J.b_top - 31) & ~(int64_t)3;
    const int sel = (int)((((J.b_top - m + 16 * g) & ~(int64_t)3) - wb) >> 2);  // 0 .. 12
    const uint32_t *bw = reinterpret_cast<const uint32_t *>(J.bd + wb) + (lane < 16 ? lane : 16);

    const int wvu = __builtin_amdgcn_readfirstlane(wv);  // wave-uniform: scalar loop control
    for (int ci = 0; ci < cpw; ++ci) {
        const int64_t t0 = ta + wvu + MFMA_WAVES * (rg * cpw + ci);
        if (t0 >= tb) break;
        const int64_t ns = uniform64((tb - t0 + 31) / 32);  // steps t = t0 + 32 k, k < ns
        // fragment slots: tile rt at step k uses fr[(rt - k) mod RT]; the loads of step k + PF
        // go into ring slot k mod PF (clamped to the last step, which stays in bounds)
        v4i fr[RT];
#pragma unroll
        for (int rt = 1; rt < RT; ++rt) fr[rt] = mfma_frag(arow, S0 + 32 * rt - t0);
        v4i pa[PF];
        uint32_t pb[PF];
        auto fetch = [&](int q, int64_t k) {
            const int64_t kk = k < ns ? k : ns - 1;
            pa[q] = mfma_frag(arow, S0 - t0 - 32 * kk);
            pb[q] = *(gu32 *)(bw - 8 * (t0 + 32 * kk));
        };
#pragma unroll
        for (int q = 0; q < PF; ++q) fetch(q, q);
        // the b-operand of step k + 1 is assembled (shuffles, realignment) while the matrix
        // operations of step k run
        v4i bop = mfma_bop(pb[0], sel, sh);
        auto step = [&](int j, int64_t k) {
            fr[(RT - j % RT) % RT] = pa[j % PF];
            fetch(j % PF, k + PF);
            // keep the loads at the head of their step (the scheduler would otherwise sink
            // them towards their uses and shorten the prefetch distance)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                acc[rt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bop, fr[(rt - j % RT + RT) % RT], acc[rt], 0, 0, 0);
            bop = mfma_bop(pb[(j + 1) % PF], sel, sh);
        };
        int64_t kb = 0;
        for (; kb + UN <= ns; kb += UN) {
#pragma unroll
            for (int j = 0; j < UN; ++j) step(j, kb + j);
        }
#pragma unroll
        for (int j = 0; j < UN - 1; ++j)
            if (kb + j < ns) step(j, kb + j);
    }
    // limb 2 a + g of output row 32 rt + m: the digits in registers 4 a .. 4 a + 3 at weights
    // 2^0, 2^8, 2^16, 2^24, exact in int64 (|digit sum| < 2^36 for a part of at most 2^17 shifts)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int a4 = 0; a4 < 4; ++a4) {
            const int64_t v = (int64_t)acc[rt][4 * a4] + (int64_t)acc[rt][4 * a4 + 1] * 256 +
                              (int64_t)acc[rt][4 * a4 + 2] * 65536 + (int64_t)acc[rt][4 * a4 + 3] * 16777216;
            const int w = 2 * a4 + g, rb = 32 * rt + m;
            D[wv][w * MFMA_ROWS + (rb ^ (8 * w))] = v;
        }
    __syncthreads();

    // limb column j of the block: its value v split as x (the low 32 bits, weight 2^0,
    // non-negative) + y (the rest, weight 2^32, signed, added in two's complement)
    unsigned long long *out = J.cols + 2 * grp * MFMA_LIMBS;
    const bool alone = J.splits * J.rgroups == 1;
    for (int j = tid; j < MFMA_LIMBS; j += MFMA_TPB) {
        const int rb = j >> 3, w = j & 7;
        const int pos = w * MFMA_ROWS + (rb ^ (8 * w));
        long long v = 0;
#pragma unroll
        for (int u = 0; u < MFMA_WAVES; ++u) v += D[u][pos];
        const unsigned long long x = (uint32_t)v, y = (unsigned long long)(v >> 32);
        if (alone) {  // the only block of its columns: plain stores, nothing cleared before
            out[2 * j] = x;
            out[2 * j + 1] = y;
        } else {
            if (x) __hip_atomic_fetch_add(out + 2 * j, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (y) __hip_atomic_fetch_add(out + 2 * j + 1, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

hipError_t launch_digitize(const Launch<DigitJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    ks_launch(digitize_kernel, dim3((unsigned)L.total_blocks), dim3(256), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_mul_mfma(const Launch<MfmaJob> &L, int rt, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    if (rt == 4)
        ks_launch(mul_mfma_kernel<4>, dim3((unsigned)L.total_blocks), dim3(MFMA_TPB), 0, s, L);
    else if (rt == 8)
        ks_launch(mul_mfma_kernel<8>, dim3((unsigned)L.total_blocks), dim3(MFMA_TPB), 0, s, L);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace ks
