// ks_mul_valu.hip -- integer products on the vector ALU (the multiplications of paper
// Sections 3.1-3.4, i.e. M(b) for KS1 and the two or four smaller products of the multipoint
// variants).
//
// Product scanning: output limb column k of A*B is sum_i a_i b_{k-i}.  A block owns a tile of
// MUL_T = 1024 consecutive columns and one split of the i range (split-K, so that even a
// single product fills the GPU); each thread owns MUL_R = 4 adjacent columns and keeps a
// 96-bit sum per column: v_mad_u64_u32 accumulates the 32x32-bit product into 64 bits and
// hands its carry to a v_addc into the top 32 bits.  Both operands stream through LDS in
// chunks of MUL_CI limbs; a_i is read as a broadcast, b as one aligned 128-bit read per four
// i steps (the four columns of a thread see a sliding window of b).
//
// Output: the 96-bit column sums are split into three 32-bit pieces landing on columns
// k, k+1, k+2, so each tile writes MUL_T + 2 int64 partial columns; the consumer
// (normalize_kernel) adds the tiles' overlaps and the splits.
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

// lo:hi (96 bits) += a * b
__device__ __forceinline__ void mac96(uint64_t &lo, uint32_t &hi, uint32_t a, uint32_t b) {
    uint64_t cc;
    asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
        "v_addc_co_u32_e64 %2, %1, 0, %2, %1"
        : "+v"(lo), "=&s"(cc), "+v"(hi)
        : "v"(a), "v"(b));
}

__global__ __launch_bounds__(MUL_TPB) void mul_valu_kernel(Launch<MulJob> L) {
    __shared__ __attribute__((aligned(16))) uint32_t sa[MUL_CI];
    __shared__ __attribute__((aligned(16))) uint32_t sb[MUL_T + MUL_CI];
    __shared__ uint64_t sspill[MUL_TPB][2];

    int64_t local;
    const MulJob J = find_job(L, (int64_t)blockIdx.x, local);
    const int tid = threadIdx.x;
    const int64_t s = local / J.ntiles;
    const int64_t t = local - s * J.ntiles;
    const int64_t k0 = t * MUL_T;

    int64_t ilo = s * J.split_len;
    if (ilo < k0 - J.nb + 1) ilo = k0 - J.nb + 1;
    if (ilo < 0) ilo = 0;
    int64_t ihi = (s + 1) * J.split_len;
    if (ihi > J.na) ihi = J.na;
    if (ihi > k0 + MUL_T) ihi = k0 + MUL_T;

    uint64_t lo[MUL_R];
    uint32_t hi[MUL_R];
#pragma unroll
    for (int r = 0; r < MUL_R; ++r) { lo[r] = 0; hi[r] = 0; }

    const int base = tid * MUL_R + MUL_CI - MUL_R;
    for (int64_t c0 = ilo; c0 < ihi; c0 += MUL_CI) {
        __syncthreads();
        sa[tid] = (c0 + tid < ihi) ? J.a[c0 + tid] : 0u;
        const int64_t bfirst = k0 - c0 - MUL_CI + 1;  // b index held in sb[0]
        for (int x = tid; x < MUL_T + MUL_CI; x += MUL_TPB) {
            int64_t bi = bfirst + x;
            sb[x] = (bi >= 0 && bi < J.nb) ? J.b[bi] : 0u;
        }
        __syncthreads();
        // E[idx] = sb[base - x0 + idx], idx in [0, 2R); column r at step x0+u uses E[R-1+r-u]
        uint4 ehi = *reinterpret_cast<const uint4 *>(&sb[base + MUL_R]);
        for (int x0 = 0; x0 < MUL_CI; x0 += MUL_R) {
            uint4 elo = *reinterpret_cast<const uint4 *>(&sb[base - x0]);
            uint4 av = *reinterpret_cast<const uint4 *>(&sa[x0]);
            uint32_t E[2 * MUL_R] = {elo.x, elo.y, elo.z, elo.w, ehi.x, ehi.y, ehi.z, ehi.w};
            uint32_t A[MUL_R] = {av.x, av.y, av.z, av.w};
#pragma unroll
            for (int u = 0; u < MUL_R; ++u)
#pragma unroll
                for (int r = 0; r < MUL_R; ++r) mac96(lo[r], hi[r], A[u], E[MUL_R - 1 + r - u]);
            ehi = elo;
        }
    }

    // split the 96-bit sums into 32-bit pieces on columns k, k+1, k+2
    int64_t own[MUL_R];
#pragma unroll
    for (int r = 0; r < MUL_R; ++r) {
        own[r] = (int64_t)(uint32_t)lo[r];
        if (r >= 1) own[r] += (int64_t)(lo[r - 1] >> 32);
        if (r >= 2) own[r] += (int64_t)hi[r - 2];
    }
    sspill[tid][0] = (lo[MUL_R - 1] >> 32) + (uint64_t)hi[MUL_R - 2];
    sspill[tid][1] = (uint64_t)hi[MUL_R - 1];
    __syncthreads();
    if (tid > 0) {
        own[0] += (int64_t)sspill[tid - 1][0];
        own[1] += (int64_t)sspill[tid - 1][1];
    }
    int64_t *out = J.part + local * MUL_TW;
#pragma unroll
    for (int r = 0; r < MUL_R; ++r) out[tid * MUL_R + r] = own[r];
    if (tid == MUL_TPB - 1) {
        out[MUL_T] = (int64_t)sspill[tid][0];
        out[MUL_T + 1] = (int64_t)sspill[tid][1];
    }
}

hipError_t launch_mul_valu(const Launch<MulJob> &L, hipStream_t s) {
    if (L.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(mul_valu_kernel, dim3((unsigned)L.total_blocks), dim3(MUL_TPB), 0, s, L);
    return hipGetLastError();
}

}  // namespace ks
