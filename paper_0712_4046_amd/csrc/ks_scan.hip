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
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

// ---- pack ------------------------------------------------------------------------------------

// Pack by scattering: each thread takes whole coefficients (coalesced loads, all independent)
// and adds their 32-bit pieces into the block's LDS limb columns; the columns before and after
// the block's range that the carry scan needs are filled the same way.
constexpr int PK_MAXW = 8;  // limbs of one input coefficient (coeff_bits <= 256)

// bits [s, s+32) of a coefficient held in registers (s may be negative: bits below 0 read 0)
__device__ __forceinline__ uint32_t reg_word(const uint32_t (&cl)[PK_MAXW], int w, uint32_t fill, int s) {
    if (s <= -32) return 0u;
    if (s < 0) return cl[0] << (-s);
    const int q = s >> 5, o = s & 31;
    uint32_t a = fill, b = fill;
#pragma unroll
    for (int t = 0; t < PK_MAXW; ++t) {
        if (t < w && t == q) a = cl[t];
        if (t < w && t == q + 1) b = cl[t];
    }
    return o ? (a >> o) | (b << (32 - o)) : a;
}

__global__ __launch_bounds__(SCAN_TPB) void pack_kernel(Launch<PackJob> L) {
    typedef BlockCarryScan<SCAN_TPB, SCAN_IPT> Scan;
    __shared__ typename Scan::Smem sm;
    __shared__ uint32_t s_ticket;
    __shared__ int64_t s_v[SCAN_BL + 3];  // s_v[x + 2] = column jb + x, x in [-2, SCAN_BL]
    if (threadIdx.x == 0) s_ticket = lb_ticket(L.ticket, L.epoch);
    for (int x = threadIdx.x; x < SCAN_BL + 3; x += SCAN_TPB) s_v[x] = 0;
    __syncthreads();
    const int64_t blk = s_ticket;
    int64_t local;
    const PackJob J = get_job(L, blk, local);
    const int tid = threadIdx.x;
    const int64_t jb = local * SCAN_BL;
    const int64_t jlo = jb - 2, jhi = jb + SCAN_BL + 1;  // columns [jlo, jhi)
    const int64_t N = J.N;
    const int bits = J.bits, w_in = J.w_in;
    const bool sgn = (J.flags & PK_SIGNED) != 0;
    // coefficients i whose bits [i N, i N + bits) meet limbs [jlo, jhi)
    const int64_t a = 32 * jlo - bits + 1;
    int64_t i0 = a <= 0 ? 0 : div_by(a + N - 1, J.N_recip);
    int64_t i1 = jhi <= 0 ? -1 : div_by(32 * jhi - 1, J.N_recip);
    if (i1 > J.L - 1) i1 = J.L - 1;
    constexpr int U = 4;  // coefficients per thread per round, loads issued together
    for (int64_t ib = i0 + tid; ib <= i1; ib += U * SCAN_TPB) {
        uint32_t cl[U][PK_MAXW];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t i = ib + (int64_t)q * SCAN_TPB;
            const int64_t ii = i <= i1 ? i : i0;
            const int64_t src = (J.flags & PK_REVERSE) ? J.L - 1 - ii : ii;
            const uint32_t *c = J.coeffs + src * w_in;
#pragma unroll
            for (int t = 0; t < PK_MAXW; ++t) {
                const uint32_t x = c[t < w_in ? t : w_in - 1];
                cl[q][t] = t < w_in ? x : 0u;
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t i = ib + (int64_t)q * SCAN_TPB;
            if (i > i1) continue;
            uint32_t top = 0;
#pragma unroll
            for (int t = 0; t < PK_MAXW; ++t) top = (t == w_in - 1) ? cl[q][t] : top;
            const uint32_t fill = (sgn && (top >> 31)) ? 0xffffffffu : 0u;
            const int64_t p = i * N;
            const int64_t w = p >> 5;
            const int r = (int)(p & 31);
            const int npieces = (bits + r + 31) >> 5;
            const bool neg = (J.flags & PK_ALTERNATE) && (i & 1);
            for (int t = 0; t < npieces; ++t) {
                const int64_t j = w + t;
                if (j < jlo || j >= jhi) continue;
                const uint32_t word = reg_word(cl[q], w_in, fill, 32 * t - r);
                int64_t piece = (sgn && t == npieces - 1) ? (int64_t)(int32_t)word : (int64_t)word;
                if (neg) piece = -piece;
                atomicAdd(reinterpret_cast<unsigned long long *>(&s_v[j - jb + 2]), (unsigned long long)piece);
            }
            if ((J.flags & PK_CHECK) && w >= jb && w < jb + SCAN_BL) {
                // range check, once per coefficient (in the block holding its lowest limb)
                bool ok;
                if (J.mod_p) {
                    ok = (((uint64_t)cl[q][1] << 32) | cl[q][0]) < J.mod_p;
                } else {
                    const int tb = bits - 32 * (w_in - 1);  // bits used in the top limb, 1..32
                    if (sgn) {
                        const int32_t sx = (int32_t)top >> (tb - 1);
                        ok = (sx == 0 || sx == -1);
                    } else {
                        ok = tb == 32 ? true : (top >> tb) == 0;
                    }
                }
                if (!ok) set_status(L.devstat, KS_DEVSTAT_RANGE);
            }
        }
    }
    __syncthreads();
    const int b0 = tid * SCAN_IPT;
    int64_t u[SCAN_IPT];
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) u[q] = u_of(s_v[b0 + q + 2], s_v[b0 + q + 1], s_v[b0 + q]);
    uint32_t out[SCAN_IPT];
    Scan::run(sm, u, out, L.status + J.block0, local, L.epoch, L.devstat);
    const int64_t j0 = jb + b0;
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q)
        if (j0 + q < J.n_out) J.out[j0 + q] = out[q];
}

// ---- normalize --------------------------------------------------------------------------------

// Each thread handles SCAN_IPT consecutive limb positions j0 .. j0+IPT-1 and needs the column
// values v at j0-2 .. j0+IPT-1.  Column j of a product is piece 0 of column-sum j, piece 1
// of j-1 and piece 2 of j-2, so the thread reads one contiguous window of column sums
// (columns j0-4 .. j0+IPT-1) plus the operand limbs of the sign corrections -- fixed-size,
// branch-free, clamped loads that are all in flight together.
constexpr int NWIN = SCAN_IPT + 4;  // column-sum window
constexpr int NV = SCAN_IPT + 2;    // column values j0-2 .. j0+IPT-1

struct TermSigns {
    bool negA[2], negB[2];
};

// v[m] += sign * (column j0 - 2 + m of the product), m in [0, NV).  Column sums come as
// three uint32 pieces per column (value j gets piece 0 of j, 1 of j-1, 2 of j-2) or as two
// uint64 per column, i.e. four uint32 words (value j gets word 0 of j, words 1 and 2 of j-1,
// word 3 of j-2).
template <int P>
__device__ __forceinline__ void column_window(const NormTerm &T, int64_t j0, int64_t (&acc)[NV]) {
    const int64_t c0 = j0 - 4;
    uint32_t x[P * NWIN];
#pragma unroll
    for (int t = 0; t < P * NWIN; ++t) {
        const int64_t col = c0 + t / P;
        const bool ok = col >= 0 && col < T.ncols;
        x[t] = T.cols[ok ? P * c0 + t : 0];
        x[t] = ok ? x[t] : 0u;
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const int w = m + 2;  // window column of position j0 - 2 + m
        if (P == 3)
            acc[m] = (int64_t)x[3 * w] + (int64_t)x[3 * (w - 1) + 1] + (int64_t)x[3 * (w - 2) + 2];
        else
            acc[m] = (int64_t)x[4 * w] + (int64_t)x[4 * (w - 1) + 1] + (int64_t)x[4 * (w - 1) + 2] +
                     (int64_t)x[4 * (w - 2) + 3];
    }
}

__device__ __forceinline__ void add_term_window(const NormTerm &T, bool negA, bool negB, int64_t j0,
                                                int64_t (&v)[NV]) {
    int64_t acc[NV];
    if (T.fmt == NORM_FMT_XY)
        column_window<4>(T, j0, acc);
    else
        column_window<3>(T, j0, acc);
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
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] += T.sign > 0 ? acc[m] : -acc[m];
}

// the slot constants 2^(off_bit0 + k period) that land in limb j
__device__ __forceinline__ int64_t offset_column(const NormJob &J, int64_t j) {
    int64_t v = 0;
    if (J.off_count > 0 && j >= 0 && 32 * j + 31 >= J.off_bit0) {
        const int64_t a = 32 * j - J.off_bit0;
        int64_t klo = a <= 0 ? 0 : div_by(a + J.off_period - 1, J.off_recip);
        int64_t khi = div_by(32 * j + 31 - J.off_bit0, J.off_recip);
        if (khi > J.off_count - 1) khi = J.off_count - 1;
        for (int64_t k = klo; k <= khi; ++k) v += (int64_t)1 << (J.off_bit0 + k * J.off_period - 32 * j);
    }
    return v;
}

// column values for positions j0-2 .. j0+IPT-1 (zero outside [0, n_in))
__device__ __forceinline__ void norm_window(const NormJob &J, const TermSigns &ts, int64_t j0, int64_t (&v)[NV]) {
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] = 0;
#pragma unroll
    for (int q = 0; q < 2; ++q)
        if (q < J.nterms) add_term_window(J.term[q], ts.negA[q], ts.negB[q], j0, v);
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const int64_t j = j0 - 2 + m;
        v[m] = (j >= 0 && j < J.n_in) ? v[m] + offset_column(J, j) : 0;
    }
}

__global__ __launch_bounds__(SCAN_TPB) void normalize_kernel(Launch<NormJob> L) {
    typedef BlockCarryScan<SCAN_TPB, SCAN_IPT> Scan;
    __shared__ typename Scan::Smem sm;
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_limb[SCAN_BL + 1];
    __shared__ int64_t s_tail[2];
    if (threadIdx.x == 0) s_ticket = lb_ticket(L.ticket, L.epoch);
    __syncthreads();
    const int64_t blk = s_ticket;
    int64_t local;
    const NormJob J = get_job(L, blk, local);
    const int tid = threadIdx.x;
    const int64_t jb = local * SCAN_BL;
    const int64_t j0 = jb + (int64_t)tid * SCAN_IPT;
    TermSigns ts;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const NormTerm &T = J.term[q];
        ts.negA[q] = q < J.nterms && (T.a[T.na - 1] >> 31) != 0;
        ts.negB[q] = q < J.nterms && (T.b[T.nb - 1] >> 31) != 0;
    }
    int64_t v[NV];
    norm_window(J, ts, j0, v);
    int64_t u[SCAN_IPT];
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) u[q] = u_of(v[q + 2], v[q + 1], v[q]);
    if (tid == SCAN_TPB - 1) {
        // the first limb of the next block is needed by the shift: its value before carries
        int64_t vn[NV];
        norm_window(J, ts, j0 + SCAN_IPT, vn);
        s_tail[0] = u_of(vn[2], vn[1], vn[0]);
    }
    uint32_t out[SCAN_IPT];
    const int kout = Scan::run(sm, u, out, L.status + J.block0, local, L.epoch, L.devstat);
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) s_limb[tid * SCAN_IPT + q] = out[q];
    if (tid == SCAN_TPB - 1) s_limb[SCAN_BL] = (uint32_t)(uint64_t)(s_tail[0] + kout);
    __syncthreads();
    // write V >> shift: output limb o takes limbs o + w and o + w + 1 (striped, coalesced)
    const int64_t w = J.shift >> 5;
    const int r = J.shift & 31;
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) {
        const int li = q * SCAN_TPB + tid;
        const int64_t o = jb + li - w;
        if (o < 0 || o >= J.n_out) continue;
        const uint32_t lo = s_limb[li];
        J.out[o] = r ? ((lo >> r) | (s_limb[li + 1] << (32 - r))) : lo;
    }
}

// ---- clearing scratch words (a kernel rather than a memset, so runs can be graph-captured) ------

__global__ __launch_bounds__(256) void fill_zero_kernel(uint64_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

hipError_t launch_fill_zero(uint64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ---- host launchers -----------------------------------------------------------------------------

hipError_t launch_pack(const Launch<PackJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)L.total_blocks), dim3(SCAN_TPB), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_normalize(const Launch<NormJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)L.total_blocks), dim3(SCAN_TPB), 0, s, L);
    return hipGetLastError();
}

}  // namespace ks
