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

__device__ __forceinline__ void check_range(const uint32_t *c, int w, int bits, bool sgn, uint64_t mod_p,
                                            uint32_t *devstat) {
    int top = bits - 32 * (w - 1);  // bits used in the top limb, 1..32
    uint32_t t = c[w - 1];
    bool ok;
    if (mod_p) {
        ok = (((uint64_t)c[1] << 32) | c[0]) < mod_p;
    } else if (sgn) {
        int32_t s = (int32_t)t >> (top - 1);
        ok = (s == 0 || s == -1);
    } else {
        ok = top == 32 ? true : (t >> top) == 0;
    }
    if (!ok) set_status(devstat, KS_DEVSTAT_RANGE);
}

__device__ int64_t pack_column(const PackJob &J, int64_t j, uint32_t *devstat) {
    if (j < 0 || j >= J.n_out) return 0;
    const int64_t N = J.N;
    const int bits = J.bits;
    const bool sgn = (J.flags & PK_SIGNED) != 0;
    int64_t ilo = div_ceil(32 * j - bits + 1, N);
    int64_t ihi = div_floor(32 * j + 31, N);
    if (ilo < 0) ilo = 0;
    if (ihi > J.L - 1) ihi = J.L - 1;
    int64_t v = 0;
    for (int64_t i = ilo; i <= ihi; ++i) {
        int64_t src = (J.flags & PK_REVERSE) ? J.L - 1 - i : i;
        const uint32_t *c = J.coeffs + src * J.w_in;
        int64_t p = i * N;
        int64_t w = p >> 5;
        int r = (int)(p & 31);
        int64_t t = j - w;
        int64_t npieces = (bits + r + 31) >> 5;
        uint32_t word = coeff_word(c, J.w_in, sgn, 32 * t - r);
        int64_t piece = (sgn && t == npieces - 1) ? (int64_t)(int32_t)word : (int64_t)word;
        if ((J.flags & PK_ALTERNATE) && (i & 1)) v -= piece; else v += piece;
        if ((J.flags & PK_CHECK) && devstat && t == 0) check_range(c, J.w_in, bits, sgn, J.mod_p, devstat);
    }
    return v;
}

__global__ __launch_bounds__(SCAN_TPB) void pack_kernel(Launch<PackJob> L) {
    typedef BlockCarryScan<SCAN_TPB, SCAN_IPT> Scan;
    __shared__ typename Scan::Smem sm;
    __shared__ uint32_t s_ticket;
    __shared__ int64_t s_last[SCAN_TPB][2];
    if (threadIdx.x == 0) s_ticket = lb_ticket(L.ticket, L.epoch);
    __syncthreads();
    const int64_t blk = s_ticket;
    int64_t local;
    const PackJob J = find_job(L, blk, local);
    const int tid = threadIdx.x;
    const int64_t j0 = local * SCAN_BL + (int64_t)tid * SCAN_IPT;

    int64_t v[SCAN_IPT];
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) v[q] = pack_column(J, j0 + q, L.devstat);
    s_last[tid][0] = v[SCAN_IPT - 2];
    s_last[tid][1] = v[SCAN_IPT - 1];
    __syncthreads();
    int64_t vm2, vm1;
    if (tid == 0) {
        vm2 = pack_column(J, j0 - 2, nullptr);
        vm1 = pack_column(J, j0 - 1, nullptr);
    } else {
        vm2 = s_last[tid - 1][0];
        vm1 = s_last[tid - 1][1];
    }
    int64_t u[SCAN_IPT];
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) {
        int64_t a1 = q >= 1 ? v[q - 1] : vm1;
        int64_t a2 = q >= 2 ? v[q - 2] : (q == 1 ? vm1 : vm2);
        u[q] = u_of(v[q], a1, a2);
    }
    uint32_t out[SCAN_IPT];
    Scan::run(sm, u, out, L.status + J.block0, local, L.epoch, L.devstat);
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q)
        if (j0 + q < J.n_out) J.out[j0 + q] = out[q];
}

// ---- normalize --------------------------------------------------------------------------------

__device__ __forceinline__ int64_t term_column(const NormTerm &T, int64_t j) {
    int64_t s = 0;
    const int64_t t = j / MUL_T;
    const int64_t x = j - t * MUL_T;
    const int64_t stride = (int64_t)T.ntiles * MUL_TW;
    for (int sp = 0; sp < T.nsplit; ++sp) {
        const int64_t *base = T.part + sp * stride;
        if (t < T.ntiles) s += base[t * MUL_TW + x];
        if (x < 2 && t >= 1 && t - 1 < T.ntiles) s += base[(t - 1) * MUL_TW + MUL_T + x];
    }
    // the multiplier works on the unsigned readings of two's-complement operands:
    // A B = Au Bu - [A<0] Bu 2^(32 na) - [B<0] Au 2^(32 nb) + [A<0][B<0] 2^(32 (na+nb))
    const bool negA = (T.a[T.na - 1] >> 31) != 0, negB = (T.b[T.nb - 1] >> 31) != 0;
    if (negA && j >= T.na && j - T.na < T.nb) s -= (int64_t)T.b[j - T.na];
    if (negB && j >= T.nb && j - T.nb < T.na) s -= (int64_t)T.a[j - T.nb];
    if (negA && negB && j == T.na + T.nb) s += 1;
    return s;
}

__device__ int64_t norm_column(const NormJob &J, int64_t j) {
    if (j < 0 || j >= J.n_in) return 0;
    int64_t v = 0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (q < J.nterms) {
            int64_t s = term_column(J.term[q], j);
            v += J.term[q].sign > 0 ? s : -s;
        }
    }
    if (J.off_count > 0) {
        int64_t klo = div_ceil(32 * j - J.off_bit0, J.off_period);
        int64_t khi = div_floor(32 * j + 31 - J.off_bit0, J.off_period);
        if (klo < 0) klo = 0;
        if (khi > J.off_count - 1) khi = J.off_count - 1;
        for (int64_t k = klo; k <= khi; ++k) v += (int64_t)1 << (J.off_bit0 + k * J.off_period - 32 * j);
    }
    return v;
}

__global__ __launch_bounds__(SCAN_TPB) void normalize_kernel(Launch<NormJob> L) {
    typedef BlockCarryScan<SCAN_TPB, SCAN_IPT> Scan;
    __shared__ typename Scan::Smem sm;
    __shared__ uint32_t s_ticket;
    __shared__ int64_t s_last[SCAN_TPB][2];
    __shared__ uint32_t s_limb[SCAN_BL + 1];
    if (threadIdx.x == 0) s_ticket = lb_ticket(L.ticket, L.epoch);
    __syncthreads();
    const int64_t blk = s_ticket;
    int64_t local;
    const NormJob J = find_job(L, blk, local);
    const int tid = threadIdx.x;
    const int64_t jb = local * SCAN_BL;
    const int64_t j0 = jb + (int64_t)tid * SCAN_IPT;

    int64_t v[SCAN_IPT];
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) v[q] = norm_column(J, j0 + q);
    s_last[tid][0] = v[SCAN_IPT - 2];
    s_last[tid][1] = v[SCAN_IPT - 1];
    __syncthreads();
    int64_t vm2, vm1;
    if (tid == 0) {
        vm2 = norm_column(J, j0 - 2);
        vm1 = norm_column(J, j0 - 1);
    } else {
        vm2 = s_last[tid - 1][0];
        vm1 = s_last[tid - 1][1];
    }
    int64_t u[SCAN_IPT];
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) {
        int64_t a1 = q >= 1 ? v[q - 1] : vm1;
        int64_t a2 = q >= 2 ? v[q - 2] : (q == 1 ? vm1 : vm2);
        u[q] = u_of(v[q], a1, a2);
    }
    uint32_t out[SCAN_IPT];
    int kout = Scan::run(sm, u, out, L.status + J.block0, local, L.epoch, L.devstat);
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) s_limb[tid * SCAN_IPT + q] = out[q];
    if (tid == SCAN_TPB - 1) {
        // the first limb of the next block, needed by the shift
        int64_t vn = norm_column(J, jb + SCAN_BL);
        s_limb[SCAN_BL] = (uint32_t)(uint64_t)(u_of(vn, v[SCAN_IPT - 1], v[SCAN_IPT - 2]) + kout);
    }
    __syncthreads();
    const int64_t w = J.shift >> 5;
    const int r = J.shift & 31;
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) {
        int64_t o = j0 + q - w;
        if (o < 0 || o >= J.n_out) continue;
        int li = tid * SCAN_IPT + q;
        uint32_t lo = s_limb[li];
        uint32_t val = r ? ((lo >> r) | (s_limb[li + 1] << (32 - r))) : lo;
        J.out[o] = val;
    }
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
