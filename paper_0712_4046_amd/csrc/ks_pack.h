// ks_pack.h -- evaluation of the inputs at the Kronecker points (the pack stage): the block
// body shared by the pack kernel and the fused pack-and-anchor launch.
#pragma once

#include "ks_device.h"

namespace ks {

// Pack by scattering: each thread takes whole coefficients (coalesced loads, all independent)
// and adds their 32-bit pieces into the block's LDS limb columns; the columns before and after
// the block's range that the carry scan needs are filled the same way.  MW bounds the
// coefficients' limbs in a launch (a launch whose inputs are all one or two limbs wide, like
// residues modulo p < 2^62, shifts two words instead of eight).
constexpr int PK_MAXW = 8;  // limbs of one input coefficient (coeff_bits <= 256)

// A block of pack job J with TPB threads (TPB * IPT limbs per block); `local` is its position
// in the job when the job has one block (else it draws a ticket).  The caller looks the job
// up in its own kernel arguments.
template <int TPB, int IPT, int MW = PK_MAXW>
__device__ __forceinline__ void pack_block(const PackJob &J, int64_t local, const LaunchCtl L) {
    constexpr int64_t BL = (int64_t)TPB * IPT;
    typedef BlockCarryScan<TPB, IPT> Scan;
    __shared__ typename Scan::Smem sm;
    __shared__ uint32_t s_ticket;
    __shared__ int64_t s_v[BL + 3];  // s_v[x + 2] = column jb + x, x in [-2, BL]
    if (J.nblocks > 1 && threadIdx.x == 0) s_ticket = (uint32_t)job_ticket(L.ctrs + J.ctr, J.nblocks);
    for (int x = threadIdx.x; x < BL + 3; x += TPB) s_v[x] = 0;
    __syncthreads();
    local = J.nblocks > 1 ? (int64_t)s_ticket : 0;  // (blocks may be interleaved across jobs)
    const int tid = threadIdx.x;
    const int64_t jb = local * BL;
    const int64_t jlo = jb - 2, jhi = jb + BL + 1;  // columns [jlo, jhi)
    const int64_t N = J.N;
    const int bits = J.bits, w_in = J.w_in;
    const bool sgn = (J.flags & PK_SIGNED) != 0;
    // coefficients i whose bits [i N, i N + bits) meet limbs [jlo, jhi)
    const int64_t a = 32 * jlo - bits + 1;
    int64_t i0 = a <= 0 ? 0 : div_by(a + N - 1, J.N_recip);
    int64_t i1 = jhi <= 0 ? -1 : div_by(32 * jhi - 1, J.N_recip);
    if (i1 > J.L - 1) i1 = J.L - 1;
    constexpr int U = 4;  // coefficients per thread per round, loads issued together
    for (int64_t ib = i0 + tid; ib <= i1; ib += U * TPB) {
        uint32_t cl[U][MW];
        const uint32_t *cq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t i = ib + (int64_t)q * TPB;
            const int64_t ii = i <= i1 ? i : i0;
            const int64_t src = (J.flags & PK_REVERSE) ? J.L - 1 - ii : ii;
            cq[q] = J.coeffs + src * w_in;
#pragma unroll
            for (int t = 0; t < MW; ++t) cl[q][t] = 0u;
        }
        // the round's coefficients with vector loads of exactly w_in words each, all in one
        // block (w_in is uniform: one scalar branch per round)
        switch (w_in) {
#define PK_LOAD(W)                                                                                  \
    case W:                                                                                         \
        if constexpr (W <= MW) {                                                                    \
            _Pragma("unroll") for (int q = 0; q < U; ++q) ldg_words<W>(cq[q], cl[q]);               \
        }                                                                                           \
        break;
            PK_LOAD(1) PK_LOAD(2) PK_LOAD(3) PK_LOAD(4) PK_LOAD(5) PK_LOAD(6) PK_LOAD(7) PK_LOAD(8)
#undef PK_LOAD
            default: break;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t i = ib + (int64_t)q * TPB;
            if (i > i1) continue;
            // the coefficient's words with their sign fill above w_in: ext[0..MW]
            uint32_t top = 0;
#pragma unroll
            for (int t = 0; t < MW; ++t) top = (t == w_in - 1) ? cl[q][t] : top;
            const uint32_t fill = (sgn && (top >> 31)) ? 0xffffffffu : 0u;
            uint32_t ext[MW + 1];
#pragma unroll
            for (int t = 0; t < MW; ++t) ext[t] = t < w_in ? cl[q][t] : fill;
            ext[MW] = fill;
            // its first bit relative to column jlo, in (-bits, 32 (BL + 3)): the low 32 bits of
            // i N and 32 jlo determine it
            const int32_t rel = (int32_t)((uint32_t)i * (uint32_t)N - ((uint32_t)jlo << 5));
            const int32_t cr = rel >> 5;  // its lowest column, relative to jlo
            const int r = rel & 31;
            const int npieces = (bits + r + 31) >> 5;  // at most MW + 1
            const uint64_t nmask = ((J.flags & PK_ALTERNATE) && (i & 1)) ? ~0ull : 0ull;
            // piece t: bits [32 t - r, 32 t - r + 32) of the coefficient, the top one read signed
#pragma unroll
            for (int t = 0; t <= MW; ++t) {
                const int32_t jr = cr + t;
                if (t < npieces && (uint32_t)jr < (uint32_t)(BL + 3)) {
                    const uint32_t word =
                        t == 0 ? ext[0] << r : (r ? __builtin_amdgcn_alignbit(ext[t], ext[t - 1], 32 - r) : ext[t]);
                    const int64_t piece = (sgn && t == npieces - 1) ? (int64_t)(int32_t)word : (int64_t)word;
                    atomicAdd(reinterpret_cast<unsigned long long *>(&s_v[jr]),
                              (unsigned long long)(((uint64_t)piece ^ nmask) - nmask));
                }
            }
            if ((J.flags & PK_CHECK) && (uint32_t)(cr - 2) < (uint32_t)BL) {
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
    const int b0 = tid * IPT;
    int64_t u[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) u[q] = u_of(s_v[b0 + q + 2], s_v[b0 + q + 1], s_v[b0 + q]);
    uint32_t out[IPT];
    Scan::run(sm, u, out, J.nblocks > 1 ? L.status + J.block0 : nullptr, local, L.epoch, L.devstat);
    const int64_t j0 = jb + b0;
#pragma unroll
    for (int q = 0; q < IPT; ++q)
        if (j0 + q < J.n_out) J.out[j0 + q] = out[q];
}

}  // namespace ks
