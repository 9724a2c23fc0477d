// ks_jobs.h -- job descriptors passed from the host planner to the libksmul kernels.
//
// Every kernel processes a list of independent jobs, one block range per job, so the same
// kernels serve a single product (a handful of jobs passed by value in the kernel
// arguments) and a batch (a job table in device memory).
#pragma once

#include <stdint.h>

namespace ks {

// device status bits (OR-ed into a word in the workspace)
constexpr uint32_t KS_DEVSTAT_RANGE = 1u;     // a coefficient was outside its declared range
constexpr uint32_t KS_DEVSTAT_CHECK = 2u;     // a reconstruction self-check failed
constexpr uint32_t KS_DEVSTAT_LOOKBACK = 4u;  // a look-back wait hit its spin limit

constexpr int MAX_INLINE_JOBS = 8;

// carry-scan kernels (pack, normalize): 256 threads x 8 limbs per block
constexpr int SCAN_TPB = 256;
constexpr int SCAN_IPT = 8;
constexpr int64_t SCAN_BL = (int64_t)SCAN_TPB * SCAN_IPT;

// vector-ALU multiplier: 256 threads x 4 columns = 1024 product limbs per tile, spilling two
// limbs into the next tile (96-bit column sums)
constexpr int MUL_TPB = 256;
constexpr int MUL_R = 4;
constexpr int MUL_T = MUL_TPB * MUL_R;
constexpr int MUL_TW = MUL_T + 2;
constexpr int MUL_CI = 256;  // i-chunk staged through LDS

constexpr int EXTRACT_TPB = 256;
constexpr int CHAIN_TPB = 64;
constexpr int ANCHOR_TPB = 256;  // four waves per anchor coefficient

enum : int32_t { PK_SIGNED = 1, PK_REVERSE = 2, PK_ALTERNATE = 4, PK_CHECK = 8 };

// operand = sum_i s_i c_{pi(i)} 2^(i N); pi reverses when PK_REVERSE, s_i = (-1)^i when
// PK_ALTERNATE; written as n_out two's-complement limbs
struct PackJob {
    const uint32_t *coeffs;
    uint32_t *out;
    int64_t L;
    int64_t n_out;
    int64_t N;
    int32_t w_in;
    int32_t bits;
    int32_t flags;
    int32_t pad;
    uint64_t mod_p;  // PK_CHECK against [0, mod_p) instead of the bit range when non-zero
    int64_t block0;
    int64_t nblocks;
};

// unsigned product of the limb arrays a (na) and b (nb); tile t of split s accumulates
// columns [t T, t T + T) over i in [s split_len, (s+1) split_len) into part[s][t][0..TW)
struct MulJob {
    const uint32_t *a;
    const uint32_t *b;
    int64_t na;
    int64_t nb;
    int64_t *part;
    int64_t split_len;
    int32_t nsplit;
    int32_t ntiles;
    int64_t block0;
    int64_t nblocks;
};

// one product read back from its partial sums, corrected for two's-complement operands
struct NormTerm {
    const int64_t *part;
    const uint32_t *a;
    const uint32_t *b;
    int64_t na;
    int64_t nb;
    int32_t nsplit;
    int32_t ntiles;
    int32_t sign;  // +1 or -1
    int32_t pad;
};

// V = sum_terms sign * product + sum_{k < off_count} 2^(off_bit0 + k off_period);
// out = V >> shift, n_out limbs; the carry scan runs over n_in limb positions
struct NormJob {
    NormTerm term[2];
    int32_t nterms;
    int32_t shift;
    int64_t off_bit0;
    int64_t off_period;
    int64_t off_count;
    uint32_t *out;
    int64_t n_out;
    int64_t n_in;
    int64_t block0;
    int64_t nblocks;
};

// output coefficient (out_first + k out_step) = slot k of src (slot bits wide) - 2^off_bit;
// written as w_out two's-complement limbs, or (mod_p != 0) as one uint64 residue
struct ExtractJob {
    const uint32_t *src;
    int64_t n_src;
    int64_t count;
    int64_t slot;
    uint32_t *out;
    int64_t out_first;
    int64_t out_step;
    int32_t w_out;
    int32_t off_bit;  // -1: nothing to subtract
    uint64_t mod_p;
    int64_t block0;
    int64_t nblocks;
};

// exact h_k + 2^off_bit for k = 2 (s K - 1) + par, s = 1 .. nseg-1 (anchors for the chains)
struct AnchorJob {
    const uint32_t *f;
    const uint32_t *g;
    int64_t lf;
    int64_t lg;
    int32_t w_in;
    int32_t sgn;
    int32_t par;
    int32_t aw;
    int64_t K;
    int64_t nseg;
    uint32_t *anchors;  // nseg * aw limbs; entry 0 unused
    int32_t off_bit;    // -1: nothing added
    int32_t pad;
    int64_t block0;
    int64_t nblocks;
};

// one parity of a four-point product: Section 3.2's reconstruction on A (digits u) and
// B (digits w, read from the top), base Y = 2^Nd, m coefficients, in segments of K
struct ChainJob {
    const uint32_t *A;
    const uint32_t *B;
    int64_t nA;
    int64_t nB;
    int64_t m;
    int64_t K;
    int64_t nseg;
    const uint32_t *anchors;
    int32_t aw;
    int32_t Nd;
    uint32_t *out;
    int64_t out_first;
    int64_t out_step;
    int32_t w_out;
    int32_t off_bit;
    uint64_t mod_p;
    int64_t block0;
    int64_t nblocks;
};

template <class J>
struct Launch {
    J jobs[MAX_INLINE_JOBS];
    const J *table;  // device table (batches); null when jobs are inline
    int64_t njobs;
    int64_t total_blocks;
    uint64_t *status;  // look-back words, one per block of the launch
    uint64_t *ticket;  // epoch-tagged block ticket counter
    uint32_t *devstat;
    uint32_t epoch;
    uint32_t pad;
};

}  // namespace ks
