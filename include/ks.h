/*
 * ks.h -- C ABI of libksmul: exact dense multiplication in Z[x] and (Z/pZ)[x] by multipoint
 * Kronecker substitution, on AMD Instinct MI355X (gfx950) GPUs.
 *
 * Method: D. Harvey, "Faster polynomial multiplication via multipoint Kronecker
 * substitution" (arXiv 0712.4046).  Problem statement (Section 3): f, g in Z[x] with
 * coefficients of length at most b bits; compute h = f g.  With e = ceil(log2 L) every
 * coefficient of h has length at most 2b + e (eq. h-inequality).  The variants reduce the
 * product to integer multiplications:
 *   KS1  -- evaluate at 2^N, N = 2b + e: one product                          (Section 3.1)
 *   NEG2 -- evaluate at +2^N and -2^N, N = b + ceil(e/2): two products, then
 *           halving, even/odd coefficients read off at 2^(2N)                   (Section 3.3)
 *   KS4  -- evaluate at +-2^N and +-2^-N (the latter through reversed inputs),
 *           N = ceil((2b+e)/4): four products, halving, and Section 3.2's
 *           carry-aware reconstruction on even and odd parts                   (Section 3.4)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Coefficient layout: a polynomial of length L with b-bit coefficients is L * W consecutive
 *   uint32 limbs, W = ceil(b / 32); coefficient i is limbs [i W, (i+1) W), little-endian.
 *   Unsigned: value in [0, 2^b), limbs above bit b zero.  KS_SIGNED: value in
 *   [-2^(b-1), 2^(b-1)) stored as two's complement sign-extended to 32 W bits (b counts the
 *   sign bit; the paper states non-negative inputs, the signed case is this library's
 *   extension).
 * Output layout: h has D = len_f + len_g - 1 coefficients of W_out = ks_out_limbs(...) limbs
 *   each, two's complement (one spare bit above the paper's 2b + e bound).
 * Pointers: f, g, h, arenas and workspaces are DEVICE pointers owned by the caller (for
 *   example torch tensors); the library never frees them.  Descriptor arrays passed to the
 *   batch planner are HOST pointers.
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue work and
 *   return; results are valid once the stream is synchronised.
 * Errors: every int-returning call returns KS_OK or a negative KS_E* code; nothing else
 *   crosses the ABI.  Argument errors are found on the host before anything is enqueued.
 *   Coefficients outside the declared range are found on the device: the call still
 *   returns KS_OK, h is unspecified, and the next status query reports KS_ERANGE.
 * Threads: calls on different streams may run concurrently from different host threads.
 *   Calls that share a stream must not be issued concurrently from several host threads.
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- variants and flags (the `variant` argument) ------------------------------------------ */
#define KS_VARIANT_AUTO 0      /* library picks KS1 / NEG2 / KS4 from its size model         */
#define KS_VARIANT_KS1 1       /* Section 3.1: one point 2^N                                 */
#define KS_VARIANT_NEG2 2      /* Section 3.3: points +-2^N                                  */
#define KS_VARIANT_RECIP2 3    /* Section 3.2: points 2^N and 2^-N (reversed polynomials),
                                  N = b + ceil(e/2), the carry-aware reconstruction at base 2^N;
                                  never chosen by KS_VARIANT_AUTO (same products as NEG2 plus the
                                  reconstruction, which the paper also finds slower)            */
#define KS_VARIANT_KS4 4       /* Section 3.4: points +-2^N, +-2^-N                          */
#define KS_P2_COMPLEX 5        /* ks_mul_poly2 only (Section 2.5): y = x^M, -x^M, i x^M over R[i],
                                  M = ceil(len_x / 2): five products in (Z/pZ)[x]            */
#define KS_P2_CUBE 6           /* ks_mul_poly2 only (Section 2.5): y = +-x^M, +-w x^M over R[w]
                                  (w a primitive cube root of unity), M = ceil(len_x / 3): eight
                                  products; needs p not divisible by 3                      */
#define KS_VARIANT_MASK 0xff
#define KS_SIGNED 0x100        /* coefficients are signed two's complement                   */
#define KS_ENGINE_VALU 0x1000  /* force the vector-ALU 32x32-bit limb multiplier            */
#define KS_ENGINE_MFMA 0x2000  /* force the int8 matrix-core (MFMA) limb multiplier          */
#define KS_ENGINE_NTT 0x4000   /* force the number-theoretic-transform multiplier (products
                                  beyond its longest transform, 2^23 terms, use the matrix cores) */
#define KS_ENGINE_ANY (KS_ENGINE_VALU | KS_ENGINE_MFMA | KS_ENGINE_NTT)
#define KS_MOD 0x10000         /* batch descriptor flag: residues mod desc.mod_p (see below) */

/* ---- status codes ------------------------------------------------------------------------- */
#define KS_OK 0
#define KS_EINVAL (-1)        /* bad argument: length < 1, bits out of [1, KS_MAX_BITS], bad variant, NULL */
#define KS_ENOMEM (-2)        /* device or host allocation failed                            */
#define KS_EHIP (-3)          /* a HIP runtime call failed                                   */
#define KS_ERANGE (-4)        /* (status query) a coefficient was outside its declared range */
#define KS_EUNSUPPORTED (-5)  /* valid request this build does not handle (e.g. no gfx950)   */
#define KS_EINTERNAL (-6)     /* (status query) an on-device self-check of the reconstruction failed */
#define KS_ESCRATCH (-7)      /* ks_mul_noalloc: the product needs more than KS_NOALLOC_SCRATCH_BYTES */

#define KS_MAX_BITS 256       /* largest coeff_bits accepted                                  */
#define KS_MAX_LEN (1LL << 24) /* largest polynomial length accepted                           */

/* Version of this ABI (major * 100 + minor). */
int32_t ks_version(void);

/* Message for a status code (static storage, never NULL). */
const char *ks_strerror(int code);

/*
 * Limbs per output coefficient for a product of lengths len_f, len_g with coeff_bits-bit
 * coefficients: ceil((2 b + e + 1) / 32), e = ceil(log2 min(len_f, len_g)) (Section 3's
 * bound 2b + e on the length of each h_i, plus a sign bit).  Returns KS_EINVAL (< 0) for
 * invalid sizes.  It takes no variant: every variant computes the same h, whose coefficients
 * the bound covers, so the output width is the same for all of them.
 */
int64_t ks_out_limbs(int64_t len_f, int64_t len_g, int32_t coeff_bits);

/*
 * h = f g in Z[x] (Section 3; variant as above).
 *   f       device, len_f * W limbs, W = ceil(coeff_bits / 32)
 *   g       device, len_g * W limbs
 *   len_f, len_g  >= 1 (unequal lengths allowed; e uses the smaller)
 *   coeff_bits    b in [1, KS_MAX_BITS]
 *   variant       KS_VARIANT_* | optional KS_SIGNED | optional KS_ENGINE_*
 *   stream        hipStream_t or NULL
 *   h       device, (len_f + len_g - 1) * ks_out_limbs(len_f, len_g, coeff_bits) limbs;
 *           must not overlap f or g
 * Scratch space comes from a library-owned pool kept per stream (grown on demand; growing
 * synchronises that stream once).  Returns KS_OK once the work is enqueued.
 */
int ks_mul(const uint32_t *f, const uint32_t *g, int64_t len_f, int64_t len_g, int32_t coeff_bits,
           int32_t variant, void *stream, uint32_t *h);

/*
 * ks_mul for callers that cannot allocate device memory: code under HIP graph capture, serving
 * loops and harnesses that forbid hipMalloc.  Arguments, layouts, results and errors are those
 * of ks_mul, and so is the work enqueued (the same kernels); the scratch comes from a fixed
 * device array of KS_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on until
 * the process ends, so the call allocates nothing (device or pinned memory) and frees nothing.
 *   Limit   a product whose scratch exceeds the array (about 63.5 MiB of operands, column sums
 *           and reconstruction buffers, and 65,536 carry-scan blocks) returns KS_ESCRATCH before
 *           anything is enqueued; ks_plan's scratch_bytes tells the size beforehand.
 *   Sharing every call on one GPU uses that GPU's array, whose contents persist between calls:
 *           calls that may overlap on one GPU (other streams or host threads) race, and the
 *           caller must order them (one stream, or events).
 *   Status  device-found errors (KS_ERANGE, KS_EINTERNAL) are reported by the next
 *           ks_stream_status on the stream of the call (with the device current).
 * The first call on a device enqueues one more small kernel that clears the array's control
 * words.
 */
#define KS_NOALLOC_SCRATCH_BYTES (64ll << 20)
int ks_mul_noalloc(const uint32_t *f, const uint32_t *g, int64_t len_f, int64_t len_g, int32_t coeff_bits,
                   int32_t variant, void *stream, uint32_t *h);

/*
 * h = f g in (Z/pZ)[x] (Section 4: lift to Z[x], multiply by a Section 3 variant, reduce).
 *   f, g    device, len_f (len_g) uint64 residues, each in [0, p)
 *   p       modulus, 2 <= p < 2^62 (any word-sized modulus of at most 62 bits; the reduction
 *           estimates quotients in double precision and needs 2 p < 2^63)
 *   variant KS_VARIANT_* | optional KS_ENGINE_* (KS_SIGNED is rejected)
 *   h       device, len_f + len_g - 1 uint64 residues in [0, p)
 * Residues >= p are reported as KS_ERANGE by the next status query.
 */
int ks_mul_mod(const uint64_t *f, const uint64_t *g, int64_t len_f, int64_t len_g, uint64_t p,
               int32_t variant, void *stream, uint64_t *h);

/*
 * h = f g in (Z/pZ)[x, y] by Kronecker substitution into (Z/pZ)[x] (Section 2).
 *   f, g    device, len_y rows of len_x uint64 residues each (row i: the coefficients of
 *           f_i(x), x^0 first, for f = sum_i f_i(x) y^i), each in [0, p)
 *   len_x, len_y  >= 1, the same for f and g (the section's assumption)
 *   p       odd modulus, 3 <= p < 2^62 (the negated points divide by 2)
 *   variant the substitution: KS_VARIANT_KS1 (standard, y = x^N, N = 2 len_x - 1, one product
 *           of length 2 len_x len_y - len_x - len_y + 1; Section 2.1), KS_VARIANT_RECIP2
 *           (y = x^N and x^-N, N = len_x, two products of length len_x len_y; Section 2.2),
 *           KS_VARIANT_NEG2 (y = +-x^N, N = len_x; Section 2.3), KS_VARIANT_KS4 (y = +-x^N,
 *           +-x^-N, N = ceil(len_x / 2), four products of length N (len_y - 1) + len_x;
 *           Section 2.4), KS_P2_COMPLEX, KS_P2_CUBE (Section 2.5's points in an extension of
 *           R: five products of length ceil(len_x / 2)(len_y - 1) + len_x, or eight of
 *           ceil(len_x / 3)(len_y - 1) + len_x; rows read off by residue mod 4 or 6),
 *           KS_VARIANT_AUTO (four points when len_x >= 2 and len_x len_y >= 24576, else the
 *           standard substitution)
 *   inner   KS_VARIANT_* | optional KS_ENGINE_* for the products in (Z/pZ)[x], which run as
 *           ks_mul_mod does (KS_SIGNED is rejected)
 *   h       device, (2 len_y - 1) rows of (2 len_x - 1) uint64 residues in [0, p)
 * Scratch (the evaluations, the univariate products) is held per stream by the library.
 * Residues >= p are reported as KS_ERANGE by the next status query; a recovery whose
 * coefficients above the product's length do not vanish as KS_EINTERNAL.
 */
int ks_mul_poly2(const uint64_t *f, const uint64_t *g, int64_t len_x, int64_t len_y, uint64_t p,
                 int32_t variant, int32_t inner, void *stream, uint64_t *h);

/*
 * Synchronise `stream`, then return and clear the device status of the library-owned pool
 * of that stream: KS_OK, KS_ERANGE or KS_EINTERNAL (KS_EHIP if the synchronisation fails).
 */
int ks_stream_status(void *stream);

/* ---- batches (many independent products in one launch sequence) --------------------------- */

/*
 * One product of a batch.  Offsets count uint32 limbs from the start of the arenas.
 * Without KS_MOD: f is len_f * W limbs, g is len_g * W limbs (W = ceil(coeff_bits / 32)),
 *   h is (len_f + len_g - 1) * ks_out_limbs(len_f, len_g, coeff_bits) limbs; flags may hold
 *   KS_SIGNED.
 * With KS_MOD: f and g are uint64 residues in [0, mod_p) (2 limbs each), h is len_f + len_g
 *   - 1 uint64 residues; coeff_bits is ignored (the bit length of mod_p is used).
 * Offsets of 64-bit data must be even.
 */
typedef struct ks_desc {
    uint64_t f_off;
    uint64_t g_off;
    uint64_t h_off;
    int32_t len_f;
    int32_t len_g;
    int32_t coeff_bits;
    int32_t flags;      /* KS_SIGNED, KS_MOD */
    uint64_t mod_p;     /* modulus, 2 <= mod_p < 2^62, when flags & KS_MOD */
} ks_desc;

typedef struct ks_batch_plan ks_batch_plan; /* opaque */
struct ks_plan_info;

/*
 * Plan a batch once: validates every descriptor (KS_EINVAL names nothing; use
 * ks_batch_plan_bad_index), sizes the scratch, orders the work, and uploads the job tables
 * to device memory owned by the plan (a synchronous upload).  `variant` applies to every
 * product (KS_VARIANT_AUTO lets the planner choose per product).  A batch of long modular
 * products of equal lengths (see KS_KARATSUBA_MIN_LIMBS) is planned as the batch of their
 * Karatsuba halves f0 g0, f1 g1 and (f0+f1)(g0+g1), h = ceil(L / 2), staged and recombined
 * mod p by two more launches inside the run (recursively while the halves qualify); the
 * result and the interface are the same.
 */
int ks_batch_plan_create(const ks_desc *descs, int64_t count, int32_t variant, ks_batch_plan **plan);
/* Index of the first descriptor rejected by the last failed ks_batch_plan_create (-1 if none). */
int64_t ks_batch_plan_bad_index(void);
/* Device scratch bytes a run of this plan needs. */
size_t ks_batch_plan_workspace_bytes(const ks_batch_plan *plan);
/* Totals over the plan's products (limb products, int8 operations, algorithmic bytes). */
int ks_batch_plan_info(const ks_batch_plan *plan, struct ks_plan_info *out);
/*
 * Enqueue the whole batch on `stream`.  Allocates nothing and copies nothing from the host,
 * so it may be captured into a hipGraph and replayed.  `workspace` (device, >= the bytes
 * above, 256-byte aligned, contents irrelevant) must not be shared by runs that may overlap.
 */
int ks_batch_run(const ks_batch_plan *plan, const uint32_t *arena_in, uint32_t *arena_out,
                 void *workspace, size_t ws_bytes, void *stream);
/* Synchronise `stream`, return and clear the status kept in `workspace` (as ks_stream_status).
   Each run starts by clearing it, so this reports the latest run on that workspace. */
int ks_batch_status(const ks_batch_plan *plan, void *workspace, void *stream);
void ks_batch_plan_destroy(ks_batch_plan *plan);

/*
 * One-shot convenience: plan, run on `workspace`, synchronise `stream` and free the plan, so
 * it returns after the batch is complete.  Not for graph capture (it uploads tables).
 */
size_t ks_batch_workspace_bytes(const ks_desc *descs, int64_t count, int32_t variant);
int ks_mul_batch(const uint32_t *arena_in, uint32_t *arena_out, const ks_desc *descs, int64_t count,
                 int32_t variant, void *workspace, size_t ws_bytes, void *stream);

/* ---- planning and measurement helpers (host only, no device work) ------------------------- */

typedef struct ks_plan_info {
    int32_t variant;          /* resolved KS_VARIANT_* */
    int32_t engine;           /* KS_ENGINE_VALU, KS_ENGINE_MFMA or KS_ENGINE_NTT (a batch: the OR of
                                 its products') */
    int32_t e;                /* ceil(log2 min(len_f, len_g)) */
    int32_t slot_bits;        /* N of the resolved variant */
    int32_t n_products;       /* 1, 2 or 4 integer products */
    int32_t out_limbs;        /* W_out */
    int64_t operand_limbs_f;  /* limbs of each evaluation of f */
    int64_t operand_limbs_g;  /* limbs of each evaluation of g */
    double limb_mults;        /* 32x32-bit partial products of the multiplier actually run */
    double schoolbook_limb_mults; /* sum over products of (limbs of a) * (limbs of b) */
    double hbm_bytes;         /* algorithmic bytes: inputs + outputs + operands + products */
    double pack_bytes;        /* per stage, algorithmic bytes moved: inputs read + operands written */
    double normalize_bytes;   /*   product column sums read once + recombined values written       */
    double finish_bytes;      /*   recombined values read + h written (extract or reconstruction)  */
    double anchor_limb_mults; /*   limb products of the reconstruction anchors (KS4)              */
    double mfma_ops;          /* int8 operations (2 per multiply-add) of the products run on the
                                 matrix cores, whose operands are balanced 8-bit digits in
                                 [-128, 127] (4 per limb and one top carry):
                                 2 * sum of (digits of a) * (digits of b) */
    double valu_limb_mults;   /* sum of (limbs of a) * (limbs of b) over the products run on the
                                 vector ALU (the rest of schoolbook_limb_mults runs on the matrix
                                 cores) */
    int64_t scratch_bytes;    /* device scratch one run needs: for ks_plan, the bytes the per-stream
                                 pool of ks_mul grows to (at least 1 MiB) for this product; for
                                 ks_batch_plan_info, the run's workspace (= ks_batch_plan_workspace_bytes) */
    double ntt_butterflies;   /* radix-2 butterflies of the products on the transform engine: three
                                 transforms of length N (two forward, one inverse) modulo each of
                                 two primes, (N / 2) log2 N butterflies each */
    int32_t ntt_k1, ntt_k2;   /* transform engine: N = 2^(k1 + k2), columns of 2^k1 and rows of 2^k2
                                 (of the first such product; 0 when none) */
} ks_plan_info;

int ks_plan(int64_t len_f, int64_t len_g, int32_t coeff_bits, int32_t variant, ks_plan_info *out);

/*
 * Per-kernel timing of the library's own launches, for roofline reports.  While enabled,
 * each launch made by ks_mul / ks_mul_mod / ks_batch_run is bracketed by HIP events on the
 * stream it is launched on; ks_profile_read synchronises those streams and returns, for
 * kernel `name`, the number of launches and their summed duration in milliseconds.  Names:
 * "pack" (with the anchors it carries), "mul_valu", "mul_mfma", "normalize", "anchor",
 * "recon", "finish", "extract", "digitize", "p2_eval", "p2_recon" (bivariate evaluation and
 * read-off or gluing), "kara" (the Karatsuba split and combination of a batch),
 * "ntt_fwd_cols", "ntt_rows", "ntt_inv_cols", "ntt_join" (the steps of the transform engine).  Returns KS_EINVAL for an unknown name.
 */
int ks_profile_enable(int32_t on);
int ks_profile_read(const char *name, int64_t *launches, double *total_ms);
int ks_profile_reset(void);

/*
 * Planner tunables (launch shapes), process-wide, read whenever a product or batch is planned;
 * a value set here overrides the environment variable of the same name, which overrides the
 * autotuner's JSON cache (the file KS_TUNING_FILE names, else $XDG_CACHE_HOME/ksmul/tuning.json
 * or $HOME/.cache/ksmul/tuning.json; read once per process, every "NAME": integer pair of a
 * known tunable taken), which overrides the built-in default.  Names and defaults:
 *   "KS_MFMA_MIN_LIMBS"  2500  both operands at least this many limbs -> matrix-core engine
 *                              (unset, the products of a batch use 1000)
 *   "KS_MFMA_BLOCKS"     0     matrix-core launch target of one product, in blocks; 0: the
 *                              launch shape of least modelled time (unset, a batch of n
 *                              products gives each max(1, 2048 / n); set, each product of a
 *                              batch aims at the value)
 *   "KS_MFMA_MIN_PART"   128   fewest block shifts the matrix-core planner gives one block
 *   "KS_MFMA_BLOCK_COST" 10    fixed cost of a matrix-core block in the launch-shape model, in
 *                              steps (MFMA_RT matrix operations of every wave)
 *   "KS_CHAIN_K"         model reconstruction segment length (0 or unset: the cost model)
 *   "KS_MUL_WAVE_MAX"    128   vector-ALU products whose shorter operand has at most this many
 *                              limbs run one wave per 128-column tile, else a block per tile
 *                              (unset, the products of a batch use 1024)
 *   "KS_MFMA_RT"         0     row tiles per matrix-core block, 4 or 8 (0: 4 for a single product
 *                              of at most 256 eight-tile row groups, else 8)
 *   "KS_SCAN_SMALL"      128   pack and recombination jobs of at most this many limbs (at most
 *                              128; in a batch at most 512 for pack and 256 for recombination,
 *                              and unset, a batch uses those) run one wave per job (0: every
 *                              job in 256-thread blocks)
 *   "KS_SCAN_BIG"        150000 a single product whose result has at least this many limbs
 *                              (D (2b + e) / 32) takes a batch's larger carry-scan blocks
 *                              (0: never)
 *   "KS_NTT_MIN_LIMBS"   40000 both operands at least this many limbs -> transform engine
 *                              (unset, the products of a batch use 12000; 0: never unless forced)
 *   "KS_KARATSUBA_MIN_LIMBS" 16384  t: a batch plan whose products are all modular with equal
 *                              lengths, whose integer operands total at least 8 t limbs and
 *                              each have at least t (2 t when the batch totals 128 t), splits
 *                              each product Karatsuba's way on the polynomials (three products
 *                              of half the length, combined mod p), and again while the halves
 *                              qualify (never when they run on the transform engine); 0: never
 * ks_tune_set returns KS_EINVAL for an unknown name or a negative value; ks_tune_get returns
 * the value in force (KS_EINVAL if unknown); ks_tune_reset clears every value set here.
 * Plans made before a change keep their shapes.  Used by paper_0712_4046_amd/autotune.py.
 */
int ks_tune_set(const char *name, int64_t value);
int ks_tune_get(const char *name, int64_t *value);
int ks_tune_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* KS_H */
