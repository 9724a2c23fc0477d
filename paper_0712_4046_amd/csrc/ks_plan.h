// ks_plan.h -- host-side plan of one product: sizes, job geometry and scratch layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <map>
#include <vector>

#include "ks_jobs.h"

struct ks_batch_plan;
struct ks_desc;

namespace ks {

int ceil_log2(int64_t x);
int64_t cdiv(int64_t a, int64_t b);

// what the caller asked for
struct Spec {
    int64_t lf, lg;
    int bits;        // b
    int w_in;        // limbs per input coefficient
    bool sgn;        // two's-complement inputs
    uint64_t mod_p;  // non-zero: inputs are residues, outputs reduced mod p
    int variant;     // KS_VARIANT_* (AUTO resolved by the planner)
    int engine;
    // launch shaping: a product planned alone takes the matrix-core launch shape of least
    // modelled time (fill_blocks = 0) and cuts reconstruction chains for latency; a product of
    // a batch shares the GPU with the rest of the batch, so it aims at a share of the blocks
    // (fill_blocks) and takes longer chain segments (fewer anchors: the batch supplies the
    // parallelism)
    int64_t fill_blocks = 0;
    bool batch = false;
    int64_t batch_count = 1;  // products planned together
};

struct PackGeom {
    int which;  // 0: f, 1: g
    int flags;  // PK_*
    int64_t L, n_out, op_off, blocks;
    bool small;  // at most small_bl(ipt) limbs: one wave
};
struct MulGeom {
    int fa, fb;  // operand (pack) indices
    int engine;  // KS_ENGINE_VALU or KS_ENGINE_MFMA
    bool wave = false;  // vector ALU, one wave per tile (short i ranges)
    int64_t na, nb, ntiles;
    int64_t ncols, cols_off, blocks;  // column sums: 3 words (vector ALU) or 4 words (matrix cores)
    // matrix-core engine: balanced 8-bit digit buffers (byte offsets in the digit region), row
    // groups of MFMA_ROWS output rows, each cut into `splits` parts of `part` block shifts,
    // each part shared by `rgroups` blocks (residue groups)
    int64_t nad = 0, nbd = 0, nA32 = 0, nB32 = 0, a_front = 0, a_len = 0, b_len = 0, b_top = 0;
    int64_t groups = 0, splits = 1, part = 0, rgroups = 1;
    int rt = 8;  // row tiles per block
    int64_t ad_off = 0, bd_off = 0;
    // transform engine: N = 2^(k1 + k2), w-bit pieces (npa, npb of them), nz convolution terms;
    // word offsets of the two transforms in the transform region (the first ends up holding the
    // terms' residues)
    int ntt_k1 = 0, ntt_k2 = 0, ntt_w = 0;
    int64_t ntt_npa = 0, ntt_npb = 0, ntt_nz = 0, ntt_xa = 0, ntt_xb = 0, ntt_cols = 0;  // + the joined columns
};
struct NormGeom {
    int nterms, prod[2], sign[2], shift;
    int64_t off_bit0, off_period, off_count, n_in, n_out, out_off, blocks;
    bool small;        // at most small_bl(ipt) limbs: one wave
    int pair = -1;     // the recombination computed in the same job (same products, other signs)
    bool merged = false;  // computed in its partner's job
};
struct ExtractGeom {
    int src;  // norm index
    int64_t count, slot, first, step, blocks;
};
struct ChainGeom {
    int A, B;  // norm indices
    int64_t m, K, nseg;
    int par;   // first output coefficient (and anchor parity)
    int step;  // output stride: 2 (a parity of the four-point product) or 1 (two-point reciprocal)
    int64_t anchor_off, anchor_blocks, chain_blocks;
    int64_t hbuf_off, finish_blocks;  // words of alpha/beta scratch; blocks of the finishing pass
};

struct Geom {
    Spec sp;
    int ipt = SCAN_IPT_SINGLE;  // limbs per thread of the carry-scan kernels
    int pack_ipt = SCAN_IPT_SINGLE;  // of the pack kernels
    int variant = 0, e = 0, w_out = 0, off = -1, nw = 0, aw = 0, chain_lds = 0;
    int64_t chain_nd = 0;  // bits of a reconstruction digit (2N four-point, N reciprocal)
    int64_t N = 0, D = 0, m0 = 0, m1 = 0, nf = 0, ng = 0;
    std::vector<PackGeom> packs;
    std::vector<MulGeom> muls;
    std::vector<NormGeom> norms;
    std::vector<ExtractGeom> extracts;
    std::vector<ChainGeom> chains;
    int64_t op_limbs = 0, col_words = 0, norm_limbs = 0, anchor_limbs = 0, digit_bytes = 0, hbuf_words = 0;
    int64_t ntt_words = 0;  // transform region (uint32 words)
    double ntt_butterflies = 0;  // butterflies of the transforms (both primes, all passes)
    int64_t pack_blocks = 0, mul_blocks = 0, norm_blocks = 0, extract_blocks = 0, anchor_blocks = 0,
            chain_blocks = 0, finish_blocks = 0;
    int64_t norm_status_extra = 0;  // look-back words of paired recombinations' second scans
    int64_t ws_ops = 0, ws_cols = 0, ws_digits = 0, ws_norms = 0, ws_anchors = 0, ws_hbuf = 0, ws_ntt = 0,
            ws_status = 0, ws_bytes = 0;
    double limb_mults = 0, school_mults = 0, hbm_bytes = 0;
    double pack_bytes = 0, normalize_bytes = 0, finish_bytes = 0, anchor_mults = 0, mfma_ops = 0;
    double valu_mults = 0;  // schoolbook limb products of the vector-ALU products
};

// device words that outlive one call: block-ticket counters (pack jobs, then normalize jobs),
// error bits, launch epoch
constexpr int CTL_CTRS = 8;  // counters per stage (a product has at most 8 pack and 4 normalize jobs)
// A stream's control words: block-ticket counters, the device status word, the launch epoch,
// and the look-back status words of its single products -- a buffer of their own that holds
// nothing but status words (cleared when allocated), so a word a launch reads is either zero or
// was published by a launch of this stream with an older epoch.  (Kept in the products' scratch,
// whose layout differs from product to product, a status word could overlie data an earlier
// product left there and read as a fresh status.)
struct Ctl {
    uint64_t *ctrs = nullptr;
    uint32_t *devstat = nullptr;
    uint32_t epoch = 0;
    uint64_t *status = nullptr;
    int64_t status_words = 0;
};

// jobs of one or many products, per stage (anchor and chain lists keyed by template parameter)
struct JobLists {
    int ipt = SCAN_IPT_SINGLE;  // limbs per thread of the carry-scan launches (as planned)
    int pack_ipt = SCAN_IPT_SINGLE;  // of the pack launches
    int mfma_rt = 8;            // row tiles per matrix-core block (the same for every product of a list)
    std::vector<PackJob> pack;
    std::vector<PackJob> pack_small;  // jobs of at most small_bl(ipt) limbs
    std::vector<MulJob> mul;
    std::vector<MulJob> mul_wave;  // small products: one wave per tile (blocks count tiles)
    std::vector<DigitJob> digit;
    std::vector<MfmaJob> mfma;
    std::vector<NttJob> ntt_f1, ntt_rows, ntt_i1;  // transform steps (forward columns per operand)
    std::vector<NttJoinJob> ntt_join;
    std::vector<NormJob> norm;
    std::vector<NormJob> norm_small;  // jobs of at most small_bl(ipt) limbs
    std::vector<ExtractJob> extract;
    std::map<int, std::vector<AnchorJob>> anchor;  // by limbs per input coefficient
    std::map<int, std::vector<ChainJob>> chain;    // by words per reconstruction digit
    std::map<int, std::vector<ChainJob>> finish;   // the same chains, one thread per coefficient
};

// a job list uploaded to the device: the table and its block -> job map
struct DevList {
    void *table = nullptr;
    uint32_t *block_job = nullptr;
};
struct DevTables {
    DevList pack, pack_small, mul, mul_wave, digit, mfma, norm, norm_small, extract, ntt_f1, ntt_rows, ntt_i1,
        ntt_join;
    std::map<int, DevList> anchor, chain, finish;
};

struct LaunchEnv {
    uint64_t *status = nullptr;
    uint64_t *ctr_pack = nullptr;  // counters indexed by PackJob::ctr
    uint64_t *ctr_norm = nullptr;  // counters indexed by NormJob::ctr
    uint32_t *devstat = nullptr;
    uintptr_t base_in = 0, base_out = 0, base_ws = 0;
};

int plan_product(const Spec &sp, Geom &G);
int64_t assign_dual_status(JobLists &JL);
void emit_jobs(const Geom &G, uintptr_t f, uintptr_t g, uintptr_t h, uintptr_t ws, JobLists &JL);
int batch_run_into(const ks_batch_plan *plan, const uint32_t *arena_in, uint32_t *arena_out, char *ws,
                   uint32_t *devstat, hipStream_t s);
int launch_lists(const JobLists &JL, const DevTables *T, const LaunchEnv &env, uint32_t epoch_pack,
                 uint32_t epoch_norm, hipStream_t s);
int run_product(const Geom &G, const uint32_t *f, const uint32_t *g, void *h, char *ws, Ctl &ctl, hipStream_t s);
int validate_spec(int64_t lf, int64_t lg, int bits, int32_t variant, bool allow_signed);
// 1 when the current device is a gfx950, else -1
int device_ok();
// synchronise s, then read and clear a device status word (KS_OK, KS_ERANGE or KS_EINTERNAL)
int read_status(uint32_t *devstat, hipStream_t s);
// the status word of ks_mul_noalloc's array on the current device (KS_OK if never used)
int noalloc_status(hipStream_t s);
// a planner tunable: the value set through ks_tune_set, else the environment, else the
// autotuner's cache file, else dflt
int env_int(const char *name, int dflt);
// counts the changes made through ks_tune_set / ks_tune_reset (cached plans compare it)
uint64_t tune_generation();
// transform length and piece width of an integer product of na x nb limbs through the
// transforms: the shortest N = 2^(k1+k2) (k1 = floor(k/2)) with a piece width w whose
// convolution fits in N terms and stays below the primes' product; false when none does
bool ntt_shape(int64_t na, int64_t nb, int min_log, int &k1, int &k2, int &w, int64_t &npa, int64_t &npb);
// R^2 / 2^k mod P_q (R = 2^32): the inverse transform's scale in the Montgomery domain
uint32_t ntt_scale(int q, int k);
// the root tables on the current device (uploaded once per device; synchronous)
int ntt_prepare();
// planner defaults of KS_NTT_MIN_LIMBS: a single product pays the transforms' four launches
// alone (measured crossing against the matrix cores: 35K-55K operand limbs), a batch shares them
constexpr int NTT_MIN_LIMBS = 40000, NTT_MIN_LIMBS_BATCH = 12000;
// planner default of KS_SCAN_BIG: a single product whose result has at least this many limbs
// (D (2b + e) / 32) takes a batch's carry-scan blocks
constexpr int SCAN_BIG_LIMBS = 150000;
// whether ks_batch_plan_create would split this batch by Karatsuba (see KS_KARATSUBA_MIN_LIMBS)
bool karatsuba_splits(const ks_desc *descs, int64_t count, int32_t variant);
// batches of modular products of equal lengths whose integer operands have at least this
// many limbs (twice as many in large batches) are split by Karatsuba on the polynomials
// (KS_KARATSUBA_MIN_LIMBS; 0: never)
constexpr int KARATSUBA_MIN_LIMBS = 16384;
// fn's launches under the stage name `name` of the launch profiler (plain launches when it is off)
hipError_t timed_launch(const char *name, hipStream_t s, const std::function<hipError_t()> &fn);

}  // namespace ks
