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

// carry-scan kernels (pack, normalize): 256 threads x IPT limbs per block, jobs of at most
// 64 IPT limbs one wave per job.  IPT = 2 for a single product (its launches are latency-bound:
// short load windows per thread), 4 for a batch (half the blocks and look-backs per job)
constexpr int SCAN_TPB = 256;
constexpr int SMALL_TPB = 64;
constexpr int SCAN_IPT_SINGLE = 2, SCAN_IPT_BATCH = 4;
// limbs per thread of a batch's pack blocks: twice the recombination's (pack keeps few values
// per limb in registers, and larger blocks pay the ticket and the look-back half as often)
constexpr int PACK_IPT_BATCH = 8;
constexpr int64_t scan_bl(int ipt) { return (int64_t)SCAN_TPB * ipt; }
constexpr int64_t small_bl(int ipt) { return (int64_t)SMALL_TPB * ipt; }

// vector-ALU multiplier: a block of MUL_WAVES waves owns MUL_T = 64 * MUL_R product columns;
// its waves take interleaved MUL_CI-long chunks of the i range and add up in LDS at the end
constexpr int MUL_WAVES = 8;
constexpr int MUL_TPB = 64 * MUL_WAVES;
constexpr int MUL_R = 2;
constexpr int MUL_T = 64 * MUL_R;
constexpr int MUL_CI = 128;

// int8 matrix-core multiplier (balanced 8-bit digits): a block of MFMA_WAVES waves owns
// RT tiles of 32 output rows (32 digits each), mfma_rows(RT) rows = mfma_limbs(RT) output
// limbs (RT = 4 or 8, chosen per plan), a
// part of the block shifts and one of rgroups groups of their residues mod 32; wave w takes
// the shifts t = t_a + c (mod 32) for the MFMA_CLASSES / rgroups residues c = w + MFMA_WAVES k
// of its group, so with parts of at most mfma_max_part(rgroups) shifts an int32 accumulator
// sees at most 4064 shifts (each adds at most 32 * 128^2 in absolute value, so the sum stays
// below 2^31)
constexpr int MFMA_WAVES = 8;
constexpr int MFMA_TPB = 64 * MFMA_WAVES;
constexpr int MFMA_CLASSES = 32 / MFMA_WAVES;
constexpr int mfma_rows(int rt) { return 32 * rt; }
constexpr int mfma_limbs(int rt) { return 256 * rt; }
constexpr int64_t mfma_max_part(int64_t rgroups) { return 4064 * 32 / (MFMA_CLASSES / rgroups); }
constexpr int64_t MFMA_PADB = 64;

constexpr int EXTRACT_TPB = 256;
constexpr int CHAIN_TPB = 64;
constexpr int FINISH_TPB = 256;
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
    uint64_t N_recip;  // division by N (see div_by)
    int32_t w_in;
    int32_t bits;
    int32_t flags;
    int32_t ctr;     // the job's block-ticket counter (see job_ticket)
    uint64_t mod_p;  // PK_CHECK against [0, mod_p) instead of the bit range when non-zero
    int64_t block0;
    int64_t nblocks;
};

// unsigned product of the limb arrays a (na) and b (nb): block t writes the 96-bit sums of
// columns [t T, t T + T) as three 32-bit pieces, cols[3 k + 0..2]
struct MulJob {
    const uint32_t *a;
    const uint32_t *b;
    int64_t na;
    int64_t nb;
    uint32_t *cols;
    int64_t block0;
    int64_t nblocks;  // = number of column tiles
};

// Balanced 8-bit digits of a limb array (n limbs: digits 0 .. 4n, see digitize_kernel) into a
// zero-padded byte buffer: out[x] = digit(x - base), or digit(base - x) when reversed (the
// Toeplitz operand is read in descending digit order) (x in [0, len)); the job's later blocks
// clear zero_len bytes at `zero` (the product's column buffer, which the matrix-core
// multiplier accumulates into)
struct DigitJob {
    const uint32_t *limbs;
    int64_t n;
    uint8_t *out;
    int64_t len;
    int64_t nd;
    int64_t base;
    int32_t reversed;
    int32_t pad;
    uint8_t *zero;
    int64_t zero_len;
    int64_t block0;
    int64_t nblocks;
};

// product of two digit buffers on the matrix cores.  Block (group, part) adds the column sums
// of limbs [group MFMA_LIMBS, (group+1) MFMA_LIMBS) over its part of the block shifts into
// cols, two uint64 per limb column (weights 2^0 and 2^32), which must start at zero
struct MfmaJob {
    const uint8_t *ad;  // a digits, a_i at ad[a_front + i]
    const uint8_t *bd;  // b digits reversed, b_i at bd[b_top - i]
    int64_t a_front;
    int64_t nA32;       // ceil(digits of a / 32)
    int64_t b_top;
    int64_t b_len;
    int64_t nB32;       // number of block shifts t
    int64_t splits;     // parts per row group
    int64_t part;       // block shifts per part (at most mfma_max_part(rgroups))
    int64_t rgroups;    // residue groups per part: 1, 2 or 4 blocks share a part
    unsigned long long *cols;
    int64_t block0;
    int64_t nblocks;
};

// Integer product through number-theoretic transforms (large operands): each operand (unsigned
// reading of its limbs) is cut into pieces of w bits, the pieces are convolved modulo two
// primes P = c 2^k + 1 below 2^31 by transforms of length N = 2^k = N1 N2 (four steps: N2
// column transforms of length N1, a twiddle, N1 row transforms of length N2; each in LDS), and
// the two residues of every convolution term are joined by the Chinese remainder theorem into
// the exact term (below P1 P2, guaranteed by the planner's choice of w).  Transforms stay in
// the order the steps leave them (rows and positions bit-reversed), which the pointwise product
// does not mind and the inverse steps undo.
constexpr int NTT_TPB = 256;
constexpr int NTT_BLOCK = 8192;   // elements a block transforms: C columns of N1, or R rows of N2
constexpr int NTT_MIN_LOG = 13, NTT_MAX_LOG = 23;  // N1 <= 2048 <= N2 <= 4096: 4 <= C <= N2
constexpr int NTT_ROOT_LOG = 23;  // root tables: powers of a root of order 2^23 of each prime
// both below 2^30 (so 4p fits in 32 bits), P0 P1 > 2^59
constexpr uint32_t NTT_P0 = 998244353u;  // 119 2^23 + 1, primitive root 3
constexpr uint32_t NTT_P1 = 897581057u;  // 107 2^23 + 1, primitive root 3

// One stage of the transforms of one operand (forward) or one product (inverse).
struct NttJob {
    const uint32_t *a;  // forward columns: the operand's limbs (unsigned reading)
    int64_t na;         // limbs of a
    int64_t np;         // pieces of a (pieces at or above np read 0)
    uint32_t *x;        // the transform, 2 N words (prime 0, then prime 1); inverse: the
                        // first operand's transform, overwritten by the product's and at last
                        // by the residues of the product's convolution terms, in order (read
                        // by the join step, NttJoinJob)
    const uint32_t *y;  // inverse rows: the second operand's transform
    int32_t k1, k2;     // N1 = 2^k1, N2 = 2^k2
    int32_t w;          // piece bits
    int32_t pad;
    uint32_t kscale[2]; // forward columns: the factor the four-step twiddles carry, per prime: R^2 / N
                        // mod P (R = 2^32) for the second operand, which with the pointwise product's
                        // R^-1 makes the inverse's scale 1 / N; R mod P (none) for the first
    int64_t block0;
    int64_t nblocks;
};

// The transform engine's last step: the two residues of every convolution term (x[m] mod P0,
// x[N + m] mod P1, m < nz) joined by the Chinese remainder theorem into the term c_m (below
// 2^62, at bit weight 2^(w m)), and the terms gathered into limb columns in the vector-ALU
// multiplier's format: column j (weight 2^(32 j)) = sum of c_m 2^(w m - 32 j) over the terms
// with floor(w m / 32) = j, as three uint32 pieces cols[3 j + 0..2] (below 2^96 for w >= 11)
struct NttJoinJob {
    const uint32_t *x;
    int64_t n;       // N: words from a term's residue mod P0 to its residue mod P1
    int64_t nz;      // terms
    int32_t w;       // piece bits
    int32_t pad;
    uint32_t *cols;  // ncols columns of three words
    int64_t ncols;
    int64_t block0;
    int64_t nblocks;
};

// column-sum formats: three uint32 pieces per column (weights 2^0, 2^32, 2^64; the vector-ALU
// multiplier and the transform engine) or two uint64 sums per column (weights 2^0, 2^32; the
// matrix-core multiplier)
enum : int32_t { NORM_FMT_PIECES = 0, NORM_FMT_XY = 1 };

// one product read back from its column sums, corrected for two's-complement operands;
// column j of the value gets piece 0 of column j, piece 1 of j-1 and piece 2 of j-2
struct NormTerm {
    const uint32_t *cols;
    const uint32_t *a;
    const uint32_t *b;
    int64_t ncols;
    int64_t na;
    int64_t nb;
    int32_t sign;  // +1 or -1
    int32_t fmt;   // NORM_FMT_PIECES or NORM_FMT_XY
};

// V = sum_terms sign * product + sum_{k < off_count} 2^(off_bit0 + k off_period);
// out = V >> shift, n_out limbs; the carry scan runs over n_in limb positions
struct NormJob {
    NormTerm term[2];
    int32_t nterms;
    int32_t shift;
    int64_t off_bit0;
    int64_t off_period;
    uint64_t off_recip;  // division by off_period (see div_by)
    int64_t off_count;
    uint32_t *out;
    int64_t n_out;
    int64_t n_in;
    int64_t ctr;  // the job's block-ticket counter (see job_ticket)
    // dual: a second value V2 = sign2[0] product0 + sign2[1] product1 + its own slot constants
    // (off_bit0_2, off_count2, same period), out2 = V2 >> shift2 (n_out2 limbs), from the same
    // column windows; its carry scan looks back through the words at status1
    int32_t dual;
    int32_t shift2;
    int32_t sign2[2];
    int64_t off_bit0_2;
    int64_t off_count2;
    uint32_t *out2;
    int64_t n_out2;
    int64_t status1;
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
    int32_t kstep;      // anchor s is coefficient kstep (s K - 1) + par
    // a second chain whose anchor s is the next coefficient, kstep (s K - 1) + par + 1 (the odd
    // chain beside the even one): computed in the same pass for s < nseg2 (0: no second chain;
    // anchors2 then repeats anchors)
    uint32_t *anchors2;
    int64_t nseg2;
    int64_t block0;
    int64_t nblocks;
};

// Section 3.2's reconstruction on A (digits u) and B (digits w, read from the top), base
// Y = 2^Nd, m coefficients, in segments of K: one parity of a four-point product (Nd = 2N,
// output coefficients par, par + 2, ...) or the whole two-point reciprocal product (Nd = N)
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
    uint32_t *hbuf;  // the chain's alpha_c, beta_c: 2 ceil(Nd/32) words per coefficient
    uint32_t *out;
    int64_t out_first;
    int64_t out_step;
    int32_t w_out;
    int32_t off_bit;
    uint64_t mod_p;
    int64_t block0;
    int64_t nblocks;
};

// floor(a / d) for 0 <= a < 2^40 and 1 <= d < 2^24 as umulhi(a, recip), recip = floor(2^64/d)+1
// (recip = 0 stands for d = 1): a reciprocal multiply instead of a 64-bit division
inline uint64_t div_recip(uint64_t d) { return d <= 1 ? 0 : (uint64_t)(~0ull / d) + 1; }

// ---- bivariate products over Z/pZ (Section 2) -------------------------------------------------

// the k evaluations of f and of g (k = 1, 2 or 4): out holds f's k polynomials of `le`
// residues, then g's; evaluation q substitutes y = (neg[q] ? -1 : 1) x^(+-n), rev[q] for the
// (normalised) reciprocal point
struct P2Eval {
    const uint64_t *f, *g;  // L_y rows of L_x residues
    uint64_t *out;
    int64_t lx, ly, n, le;
    uint64_t p;
    int32_t k, pad;
    int32_t neg[4], rev[4];
    uint32_t *devstat;
};

// one side of the recovery: value(pos) = x[pos + off] (comb 0) or (x +- y)[pos + off] / 2
// (comb +-1), zero outside [0, len)
struct P2Side {
    const uint64_t *x, *y;
    int64_t len, off;
    int32_t comb, pad;
};

// h_k[c] = (k odd ? odd : even)(k n + c), rows x width residues
struct P2Readoff {
    P2Side even, odd;
    uint64_t *out;
    int64_t rows, width, n;
    uint64_t p;
};

// gluing of `count` polynomials at block m from A (forward) and B (reversed); u_j goes to
// output row row0 + j rstep (width residues per row); sums: nchunks x 4m chunk totals, chunks
// of P2_CHUNK steps.  One launch glues up to two parts (the four-point even and odd parts).
constexpr int P2_CHUNK = 8;
struct P2GluePart {
    P2Side A, B;
    uint64_t *sums;
    int64_t count, row0, rstep, nchunks;
};
struct P2Glue {
    P2GluePart part[2];
    int32_t nparts, pad;
    uint64_t *out;
    int64_t m, width;
    uint64_t p;
    uint32_t *devstat;
};

// Section 2.5's evaluation points in an extension S of R = Z/pZ (S = R[i] or R[w], w a
// primitive cube root of unity): out holds np polynomials of `le` residues for f, then the same
// for g; polynomial q is sum_i coef[q][i mod period] f_i(x) x^(i m) with small integer
// coefficients (the real and second parts of z^i for the points z x^m, and their sums for the
// ring products' middle terms)
struct P2ExtEval {
    const uint64_t *f, *g;
    uint64_t *out;
    int64_t lx, ly, m, le;
    uint64_t p;
    int32_t np, period;
    int8_t coef[8][8];
    uint32_t *devstat;
};

// Recovery from the products (product q at prod + q lh, lh = 2 le - 1 residues): the inverse
// transform of length 4 (complex points) or 6 (cube roots) per position, row j of h read off
// the class j mod 4 (or 6) at x^(j m); `inv` is 4^-1 (or 6^-1) mod p
struct P2ExtReadoff {
    const uint64_t *prod;
    uint64_t *out;
    int64_t lh, rows, width, m;
    uint64_t p, inv;
    int32_t cube, pad;
};

// One modular product of a batch split at the polynomial level (Karatsuba): f = f0 + x^h f1,
// g = g0 + x^h g1 with h = ceil(L / 2) (f1, g1 zero-padded to h terms), staged as six arrays
// of h residues [f0 f1 f0+f1 g0 g1 g0+g1] from residue `sub_in` of the staging arena; the three
// products f0 g0, f1 g1, (f0+f1)(g0+g1), 2h - 1 residues each, come back in that order from
// residue `sub_out` of the product arena, and
// f g = f0 g0 + x^h ((f0+f1)(g0+g1) - f0 g0 - f1 g1) + x^(2h) f1 g1.
struct KaraProd {
    uint64_t f_off, g_off, h_off;  // uint32-word offsets in the caller's arenas
    int64_t L, h;
    int64_t sub_in, sub_out;
    uint64_t p;
};

// Pointer fields of a job are addresses relative to a base: inputs (f, g) to base_in,
// outputs (h) to base_out, scratch to base_ws.  Single products pass absolute addresses with
// zero bases; batch plans store byte offsets once and the bases arrive with each run.
template <class J>
struct Launch {
    J jobs[MAX_INLINE_JOBS];
    const J *table;              // device job table (batches); null when jobs are inline
    const uint32_t *block_job;   // device map block -> job index (with table)
    int64_t njobs;
    int64_t total_blocks;
    uint64_t *status;  // look-back words, one per block of the launch
    uint64_t *ctrs;    // block-ticket counters of the carry-scan jobs (see job_ticket)
    uint32_t *devstat;
    uint32_t epoch;
    uint32_t pad;
    uintptr_t base_in, base_out, base_ws;
};

}  // namespace ks
