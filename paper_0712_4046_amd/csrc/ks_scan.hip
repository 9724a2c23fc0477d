// ks_scan.hip -- the two carry-scan stages of the pipeline.
//
// pack_kernel      Evaluation of the inputs at the Kronecker points (paper Sections 3.1,
//                  3.3, 3.4): operand = sum_i s_i c_i 2^(i N), with s_i = (-1)^i for the
//                  negated points and the coefficient order reversed for the reciprocal
//                  points.  Each limb column sums the (signed) 32-bit pieces of every
//                  coefficient that overlaps it -- in Section 3.4 several do, because
//                  N < b -- and the carry scan turns the columns into two's-complement limbs.
//                  The job flagged PK_CHECK also validates each coefficient's range.
// normalize_kernel Recombination of products (Sections 3.3, 3.4): sum_terms +-H plus an
//                  optional constant slot pattern, carry-resolved, then shifted right
//                  exactly (the halvings (H1+H2)/2 and (H1-H2)/2^(N+1)).
#include "ks_anchor.h"
#include "ks_device.h"
#include "ks_launch.h"
#include "ks_pack.h"

namespace ks {

// ---- pack ------------------------------------------------------------------------------------

template <int IPT, int MW = PK_MAXW>
__global__ __launch_bounds__(SCAN_TPB) void pack_kernel(Launch<PackJob> L) {
    int64_t local;
    const PackJob J = get_job(L, (int64_t)blockIdx.x, local);
    pack_block<SCAN_TPB, IPT, MW>(J, local, ctl_of(L));
}

// jobs of at most small_bl(IPT) limbs (one block each): one wave per job
template <int IPT, int MW = PK_MAXW>
__global__ __launch_bounds__(SMALL_TPB) void pack_small_kernel(Launch<PackJob> L) {
    int64_t local;
    const PackJob J = get_job(L, (int64_t)blockIdx.x, local);
    pack_block<SMALL_TPB, IPT, MW>(J, local, ctl_of(L));
}

// Pack and anchors in one launch: anchors read only the inputs and so run beside the packing.
// In a batch the anchor blocks, fewer and longer (a dot product over the inputs each), go
// first (blocks [0, anchor blocks)) and the short pack blocks fill in around them; a single
// product, bound by its pack's look-back chain, dispatches its pack blocks first.  (Pack
// blocks wait only on pack blocks that drew earlier tickets, anchor blocks on nothing.)
static_assert(SCAN_TPB == ANCHOR_TPB, "pack and anchor blocks share one launch");
template <int W, int IPT, int MW = PK_MAXW>
__global__ __launch_bounds__(SCAN_TPB) void pack_anchor_kernel(Launch<PackJob> Lp, Launch<AnchorJob> La) {
    int64_t local;
    constexpr bool AFIRST = IPT == PACK_IPT_BATCH;
    const int64_t pb = AFIRST ? (int64_t)blockIdx.x - La.total_blocks : (int64_t)blockIdx.x;
    const int64_t ab = AFIRST ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - Lp.total_blocks;
    if (pb >= 0 && pb < Lp.total_blocks) {
        const PackJob J = get_job(Lp, pb, local);
        pack_block<SCAN_TPB, IPT, MW>(J, local, ctl_of(Lp));
    } else {
        // a product's anchors re-read its inputs: keep them on one XCD (xcd_block)
        const AnchorJob J = get_job(La, xcd_block(ab, La.total_blocks), local);
        if (J.nseg2 > 0)
            anchor_pair_block<W>(J, local);
        else
            anchor_block<W>(J, local);
    }
}

// ---- normalize --------------------------------------------------------------------------------

// Each thread handles IPT consecutive limb positions j0 .. j0+IPT-1 and needs the column
// values v at j0-2 .. j0+IPT-1.  Column j of a product is piece 0 of column-sum j, piece 1
// of j-1 and piece 2 of j-2, so the thread reads one contiguous window of column sums
// (columns j0-4 .. j0+IPT-1) plus the operand limbs of the sign corrections -- fixed-size,
// branch-free, clamped loads that are all in flight together.
// (columns j0-4 .. j0+IPT-1: IPT + 4 of them; column values j0-2 .. j0+IPT-1: IPT + 2)

struct TermSigns {
    bool negA[2], negB[2];
};

// v[m] += sign * (column j0 - 2 + m of the product), m in [0, IPT + 2).  Column sums come as
// three uint32 pieces per column (value j gets piece 0 of j, 1 of j-1, 2 of j-2) or as two
// uint64 per column, x + y 2^32 with x non-negative and y signed (the matrix cores' balanced
// digits give signed partial sums), i.e. four uint32 words (value j gets word 0 of j, words 1
// and 2 of j-1, word 3 of j-2 read as a signed 32-bit value).
template <int P, int IPT>
__device__ __forceinline__ void column_window(const NormTerm &T, int64_t j0, int64_t (&acc)[IPT + 2]) {
    constexpr int NWIN = IPT + 4, NV = IPT + 2;
    const int64_t c0 = j0 - 4;
    uint32_t x[P * NWIN];
    // one vector load per column (clamped address, zeroed outside the product)
#pragma unroll
    for (int w = 0; w < NWIN; ++w) {
        const int64_t col = c0 + w;
        const bool ok = col >= 0 && col < T.ncols;
        ldg_words<P>(T.cols + P * (ok ? col : 0), x + P * w);
#pragma unroll
        for (int t = 0; t < P; ++t) x[P * w + t] = ok ? x[P * w + t] : 0u;
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const int w = m + 2;  // window column of position j0 - 2 + m
        if (P == 3)
            acc[m] = (int64_t)x[3 * w] + (int64_t)x[3 * (w - 1) + 1] + (int64_t)x[3 * (w - 2) + 2];
        else
            acc[m] = (int64_t)x[4 * w] + (int64_t)x[4 * (w - 1) + 1] + (int64_t)x[4 * (w - 1) + 2] +
                     (int64_t)(int32_t)x[4 * (w - 2) + 3];  // y is signed (balanced digits)
    }
}

// the window of one product (signs of its operands corrected, its own sign not applied)
template <int IPT>
__device__ __forceinline__ void term_window(const NormTerm &T, bool negA, bool negB, int64_t j0,
                                            int64_t (&acc)[IPT + 2]) {
    constexpr int NV = IPT + 2;
    if (T.fmt == NORM_FMT_XY)
        column_window<4, IPT>(T, j0, acc);
    else
        column_window<3, IPT>(T, j0, acc);
    // the multiplier works on the unsigned readings of two's-complement operands:
    // A B = Au Bu - [A<0] Bu 2^(32 na) - [B<0] Au 2^(32 nb) + [A<0][B<0] 2^(32 (na+nb))
    if (negA) {
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            const int64_t ib = j0 - 2 + m - T.na;
            const bool ok = ib >= 0 && ib < T.nb;
            const uint32_t bv = T.b[ok ? ib : 0];
            acc[m] -= ok ? (int64_t)bv : 0;
        }
    }
    if (negB) {
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            const int64_t ia = j0 - 2 + m - T.nb;
            const bool ok = ia >= 0 && ia < T.na;
            const uint32_t av = T.a[ok ? ia : 0];
            acc[m] -= ok ? (int64_t)av : 0;
        }
    }
    if (negA && negB) {
#pragma unroll
        for (int m = 0; m < NV; ++m) acc[m] += (j0 - 2 + m == T.na + T.nb) ? 1 : 0;
    }
}

template <int IPT>
__device__ __forceinline__ void add_term_window(const NormTerm &T, bool negA, bool negB, int64_t j0,
                                                int64_t (&v)[IPT + 2]) {
    constexpr int NV = IPT + 2;
    int64_t acc[NV];
    term_window<IPT>(T, negA, negB, j0, acc);
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] += T.sign > 0 ? acc[m] : -acc[m];
}

// the slot constants 2^(bit0 + k period), k < count, that land in limb j
__device__ __forceinline__ int64_t offset_column(const NormJob &J, int64_t j, int64_t bit0, int64_t count) {
    int64_t v = 0;
    if (count > 0 && j >= 0 && 32 * j + 31 >= bit0) {
        const int64_t a = 32 * j - bit0;
        int64_t klo = a <= 0 ? 0 : div_by(a + J.off_period - 1, J.off_recip);
        int64_t khi = div_by(32 * j + 31 - bit0, J.off_recip);
        if (khi > count - 1) khi = count - 1;
        for (int64_t k = klo; k <= khi; ++k) v += (int64_t)1 << (bit0 + k * J.off_period - 32 * j);
    }
    return v;
}
__device__ __forceinline__ int64_t offset_column(const NormJob &J, int64_t j) {
    return offset_column(J, j, J.off_bit0, J.off_count);
}

// column values for positions j0-2 .. j0+IPT-1 (zero outside [0, n_in))
template <int IPT>
__device__ __forceinline__ void norm_window(const NormJob &J, const TermSigns &ts, int64_t j0, int64_t (&v)[IPT + 2]) {
    constexpr int NV = IPT + 2;
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] = 0;
#pragma unroll
    for (int q = 0; q < 2; ++q)
        if (q < J.nterms) add_term_window<IPT>(J.term[q], ts.negA[q], ts.negB[q], j0, v);
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const int64_t j = j0 - 2 + m;
        v[m] = (j >= 0 && j < J.n_in) ? v[m] + offset_column(J, j) : 0;
    }
}

// both values of a dual job: V = sign[0] P0 + sign[1] P1 + its slot constants and V2 =
// sign2[0] P0 + sign2[1] P1 + its own, from one read of each product's window
template <int IPT>
__device__ __forceinline__ void norm_window_dual(const NormJob &J, const TermSigns &ts, int64_t j0,
                                                 int64_t (&v0)[IPT + 2], int64_t (&v1)[IPT + 2]) {
    constexpr int NV = IPT + 2;
    int64_t a0[NV], a1[NV];
    term_window<IPT>(J.term[0], ts.negA[0], ts.negB[0], j0, a0);
    term_window<IPT>(J.term[1], ts.negA[1], ts.negB[1], j0, a1);
    const int s0 = J.term[0].sign, s1 = J.term[1].sign, t0 = J.sign2[0], t1 = J.sign2[1];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const int64_t j = j0 - 2 + m;
        const bool in = j >= 0 && j < J.n_in;
        const int64_t x = (s0 > 0 ? a0[m] : -a0[m]) + (s1 > 0 ? a1[m] : -a1[m]);
        const int64_t y = (t0 > 0 ? a0[m] : -a0[m]) + (t1 > 0 ? a1[m] : -a1[m]);
        v0[m] = in ? x + offset_column(J, j) : 0;
        v1[m] = in ? y + offset_column(J, j, J.off_bit0_2, J.off_count2) : 0;
    }
}

// A block of recombination job J with TPB threads (TPB * IPT limbs per block); the caller
// looks the job up in its own kernel arguments.
template <int TPB, int IPT, bool DUAL = true>
__device__ __forceinline__ void normalize_block(const NormJob &J, int64_t local, const LaunchCtl L) {
    constexpr int64_t BL = (int64_t)TPB * IPT;
    constexpr int NV = IPT + 2;
    typedef BlockCarryScan<TPB, IPT> Scan;
    __shared__ typename Scan::Smem sm;
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_limb[BL + 1];
    __shared__ int64_t s_tail[2];
    if (J.nblocks > 1 && threadIdx.x == 0) s_ticket = (uint32_t)job_ticket(L.ctrs + J.ctr, J.nblocks);
    __syncthreads();
    local = J.nblocks > 1 ? (int64_t)s_ticket : 0;  // (blocks may be interleaved across jobs)
    const int tid = threadIdx.x;
    const int64_t jb = local * BL;
    const int64_t j0 = jb + (int64_t)tid * IPT;
    TermSigns ts;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const NormTerm &T = J.term[q];
        ts.negA[q] = q < J.nterms && (T.a[T.na - 1] >> 31) != 0;
        ts.negB[q] = q < J.nterms && (T.b[T.nb - 1] >> 31) != 0;
    }
    // scan u (this block's pre-carry values; tail: the next block's first one) and write
    // V >> shift: output limb o takes limbs o + w and o + w + 1 (striped, coalesced)
    auto scan_out = [&](const int64_t (&u)[IPT], int64_t tail, uint64_t *st, uint32_t *dst, int64_t n_out,
                        int shift) {
        uint32_t out[IPT];
        const int kout = Scan::run(sm, u, out, st, local, L.epoch, L.devstat);
#pragma unroll
        for (int q = 0; q < IPT; ++q) s_limb[tid * IPT + q] = out[q];
        if (tid == TPB - 1) s_limb[BL] = (uint32_t)(uint64_t)(tail + kout);
        __syncthreads();
        const int64_t w = shift >> 5;
        const int r = shift & 31;
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int li = q * TPB + tid;
            const int64_t o = jb + li - w;
            if (o < 0 || o >= n_out) continue;
            const uint32_t lo = s_limb[li];
            dst[o] = r ? ((lo >> r) | (s_limb[li + 1] << (32 - r))) : lo;
        }
    };
    int64_t v[NV];
    int64_t u[IPT];
    if (!DUAL || !J.dual) {
        norm_window<IPT>(J, ts, j0, v);
#pragma unroll
        for (int q = 0; q < IPT; ++q) u[q] = u_of(v[q + 2], v[q + 1], v[q]);
        if (tid == TPB - 1) {
            // the first limb of the next block is needed by the shift: its value before carries
            int64_t vn[NV];
            norm_window<IPT>(J, ts, j0 + IPT, vn);
            s_tail[0] = u_of(vn[2], vn[1], vn[0]);
        }
        scan_out(u, s_tail[0], J.nblocks > 1 ? L.status + J.block0 : nullptr, J.out, J.n_out, J.shift);
        return;
    }
    int64_t v2[NV], u2[IPT];
    norm_window_dual<IPT>(J, ts, j0, v, v2);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        u[q] = u_of(v[q + 2], v[q + 1], v[q]);
        u2[q] = u_of(v2[q + 2], v2[q + 1], v2[q]);
    }
    if (tid == TPB - 1) {
        int64_t vn[NV], vn2[NV];
        norm_window_dual<IPT>(J, ts, j0 + IPT, vn, vn2);
        s_tail[0] = u_of(vn[2], vn[1], vn[0]);
        s_tail[1] = u_of(vn2[2], vn2[1], vn2[0]);
    }
    if constexpr (!DUAL) return;
    scan_out(u, s_tail[0], J.nblocks > 1 ? L.status + J.block0 : nullptr, J.out, J.n_out, J.shift);
    __syncthreads();  // s_limb and the scan's shared words are reused
    scan_out(u2, s_tail[1], J.nblocks > 1 ? L.status + J.status1 : nullptr, J.out2, J.n_out2, J.shift2);
}

// at least five waves per SIMD: the register budget (96) that keeps the column window's loads
// in flight without spilling, and one more wave than the unconstrained allocation (100)
// DUAL: the launch has paired jobs (the single-value kernel keeps its own register allocation)
template <int IPT, bool DUAL = false>
__global__ __launch_bounds__(SCAN_TPB, 5) void normalize_kernel(Launch<NormJob> L) {
    int64_t local;
    const NormJob J = get_job(L, (int64_t)blockIdx.x, local);
    normalize_block<SCAN_TPB, IPT, DUAL>(J, local, ctl_of(L));
}

template <int IPT>
__global__ __launch_bounds__(SMALL_TPB, 5) void normalize_small_kernel(Launch<NormJob> L) {
    int64_t local;
    const NormJob J = get_job(L, (int64_t)blockIdx.x, local);
    normalize_block<SMALL_TPB, IPT, false>(J, local, ctl_of(L));
}

// ---- clearing scratch words (a kernel rather than a memset, so runs can be graph-captured) ------

__global__ __launch_bounds__(256) void fill_zero_kernel(uint64_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

hipError_t launch_fill_zero(uint64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    ks_launch(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ---- host launchers -----------------------------------------------------------------------------

// the instantiation of a scan kernel for the plan's limbs per thread (2 or 4)
#define KS_SCAN_IPT(ipt, K, ...)                            \
    do {                                                    \
        if ((ipt) == SCAN_IPT_BATCH)                        \
            ks_launch(K<SCAN_IPT_BATCH>, __VA_ARGS__);      \
        else                                                \
            ks_launch(K<SCAN_IPT_SINGLE>, __VA_ARGS__);     \
    } while (0)

// the pack kernels of a batch (PACK_IPT_BATCH limbs per thread) or of a single product
#define KS_PACK_IPT(ipt, K, ...)                            \
    do {                                                    \
        if ((ipt) == PACK_IPT_BATCH)                        \
            ks_launch(K<PACK_IPT_BATCH>, __VA_ARGS__);      \
        else                                                \
            ks_launch(K<SCAN_IPT_SINGLE>, __VA_ARGS__);     \
    } while (0)

hipError_t launch_pack(const Launch<PackJob> &L, int ipt, int pack_w, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    const dim3 g((unsigned)L.total_blocks), b(SCAN_TPB);
    const bool batch = ipt == PACK_IPT_BATCH;
    if (pack_w <= 2) {
        if (batch)
            ks_launch(pack_kernel<PACK_IPT_BATCH, 2>, g, b, 0, s, L);
        else
            ks_launch(pack_kernel<SCAN_IPT_SINGLE, 2>, g, b, 0, s, L);
    } else if (pack_w <= 4) {
        if (batch)
            ks_launch(pack_kernel<PACK_IPT_BATCH, 4>, g, b, 0, s, L);
        else
            ks_launch(pack_kernel<SCAN_IPT_SINGLE, 4>, g, b, 0, s, L);
    } else {
        KS_PACK_IPT(ipt, pack_kernel, g, b, 0, s, L);
    }
    return hipGetLastError();
}

template <int IPT>
static hipError_t pack_anchor_w(const Launch<PackJob> &Lp, const Launch<AnchorJob> &La, int w_in, int pack_w,
                                hipStream_t s) {
    dim3 g((unsigned)(Lp.total_blocks + La.total_blocks)), b(SCAN_TPB);
    if (pack_w <= 2 && w_in <= 2) {  // every input one or two limbs wide (residues)
        if (w_in == 1)
            ks_launch(pack_anchor_kernel<1, IPT, 2>, g, b, 0, s, Lp, La);
        else
            ks_launch(pack_anchor_kernel<2, IPT, 2>, g, b, 0, s, Lp, La);
        return hipGetLastError();
    }
    if (pack_w <= 4 && w_in <= 4) {  // at most four limbs (coefficients of up to 128 bits)
        switch (w_in) {
            case 1: ks_launch(pack_anchor_kernel<1, IPT, 4>, g, b, 0, s, Lp, La); break;
            case 2: ks_launch(pack_anchor_kernel<2, IPT, 4>, g, b, 0, s, Lp, La); break;
            case 3: ks_launch(pack_anchor_kernel<3, IPT, 4>, g, b, 0, s, Lp, La); break;
            default: ks_launch(pack_anchor_kernel<4, IPT, 4>, g, b, 0, s, Lp, La); break;
        }
        return hipGetLastError();
    }
    switch (w_in) {
        case 1: ks_launch(pack_anchor_kernel<1, IPT>, g, b, 0, s, Lp, La); break;
        case 2: ks_launch(pack_anchor_kernel<2, IPT>, g, b, 0, s, Lp, La); break;
        case 3: ks_launch(pack_anchor_kernel<3, IPT>, g, b, 0, s, Lp, La); break;
        case 4: ks_launch(pack_anchor_kernel<4, IPT>, g, b, 0, s, Lp, La); break;
        case 5: ks_launch(pack_anchor_kernel<5, IPT>, g, b, 0, s, Lp, La); break;
        case 6: ks_launch(pack_anchor_kernel<6, IPT>, g, b, 0, s, Lp, La); break;
        case 7: ks_launch(pack_anchor_kernel<7, IPT>, g, b, 0, s, Lp, La); break;
        case 8: ks_launch(pack_anchor_kernel<8, IPT>, g, b, 0, s, Lp, La); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_anchor(const Launch<PackJob> &Lp, const Launch<AnchorJob> &La, int w_in, int ipt,
                              int pack_w, hipStream_t s) {
    if (La.total_blocks <= 0) return launch_pack(Lp, ipt, pack_w, s);
    return ipt == PACK_IPT_BATCH ? pack_anchor_w<PACK_IPT_BATCH>(Lp, La, w_in, pack_w, s)
                                 : pack_anchor_w<SCAN_IPT_SINGLE>(Lp, La, w_in, pack_w, s);
}

hipError_t launch_pack_small(const Launch<PackJob> &L, int ipt, int pack_w, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    const dim3 g((unsigned)L.total_blocks), b(SMALL_TPB);
    const bool batch = ipt == PACK_IPT_BATCH;
    if (pack_w <= 2) {
        if (batch)
            ks_launch(pack_small_kernel<PACK_IPT_BATCH, 2>, g, b, 0, s, L);
        else
            ks_launch(pack_small_kernel<SCAN_IPT_SINGLE, 2>, g, b, 0, s, L);
    } else if (pack_w <= 4) {
        if (batch)
            ks_launch(pack_small_kernel<PACK_IPT_BATCH, 4>, g, b, 0, s, L);
        else
            ks_launch(pack_small_kernel<SCAN_IPT_SINGLE, 4>, g, b, 0, s, L);
    } else {
        KS_PACK_IPT(ipt, pack_small_kernel, g, b, 0, s, L);
    }
    return hipGetLastError();
}

hipError_t launch_normalize_small(const Launch<NormJob> &L, int ipt, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    KS_SCAN_IPT(ipt, normalize_small_kernel, dim3((unsigned)L.total_blocks), dim3(SMALL_TPB), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_normalize(const Launch<NormJob> &L, int ipt, bool dual, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    const dim3 g((unsigned)L.total_blocks), b(SCAN_TPB);
    if (dual) {
        if (ipt == SCAN_IPT_BATCH)
            ks_launch(normalize_kernel<SCAN_IPT_BATCH, true>, g, b, 0, s, L);
        else
            ks_launch(normalize_kernel<SCAN_IPT_SINGLE, true>, g, b, 0, s, L);
    } else {
        KS_SCAN_IPT(ipt, normalize_kernel, g, b, 0, s, L);
    }
    return hipGetLastError();
}

}  // namespace ks
