// ks_batch.cpp -- many independent products planned once and run as one launch sequence.
//
// Every product of a batch is planned like a single product (ks_api.cpp); their jobs are
// concatenated per stage, so each stage is one kernel launch over all products (one per
// template parameter for the anchor and chain stages).  Job tables and block -> job maps live
// in device memory owned by the plan; pointers in them are byte offsets from the run's
// arenas and workspace.  A run allocates nothing and copies nothing from the host: it clears
// the look-back words with a kernel and launches the stages, so it can be graph-captured.
//
// Workspace layout (bytes): [0, 8) device status word, [64, 64 + 8 S) look-back status words,
// then one block-ticket counter per pack job and per normalize job (8 bytes each), then each
// product's scratch, 256-byte aligned.  Every run clears everything before the scratch first,
// so a fresh (uninitialised) workspace needs no set-up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/ks.h"
#include "ks_jobs.h"
#include "ks_launch.h"
#include "ks_plan.h"

namespace ks {

int read_status(uint32_t *devstat, hipStream_t s);
int device_ok();
int bitlen_u64(uint64_t x);

static thread_local int64_t g_bad_index = -1;

static int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// A job list and its block -> job map on the device.  interleave: the carry-scan stages, whose
// blocks draw their positions from their job's ticket counter and look back over their job's
// status words -- the launch's blocks go round-robin over the jobs (the first block of every
// job, then the second, ...), so that the blocks running at one time draw from many counters
// and poll many status lines.  Taken in job order, the ~1300 blocks resident at once belonged
// to a handful of jobs, and their same-address atomics serialised: the 64-product modular
// batch's pack and recombination spent about half their time there.
template <class J>
static int upload(const std::vector<J> &jobs, DevList &d, std::vector<void *> &allocs, bool interleave = false) {
    if (jobs.empty()) return KS_OK;
    const int64_t nb = jobs.back().block0 + jobs.back().nblocks;
    std::vector<uint32_t> map((size_t)nb);
    if (interleave) {
        std::vector<size_t> live(jobs.size());
        for (size_t i = 0; i < jobs.size(); ++i) live[i] = i;
        int64_t g = 0;
        for (int64_t r = 0; !live.empty(); ++r) {
            size_t keep = 0;
            for (size_t i : live)
                if (jobs[i].nblocks > r) {
                    map[(size_t)g++] = (uint32_t)i;
                    if (jobs[i].nblocks > r + 1) live[keep++] = i;
                }
            live.resize(keep);
        }
        if (g != nb) return KS_EINTERNAL;  // the list's blocks must be numbered without gaps
    } else {
        for (size_t i = 0; i < jobs.size(); ++i)
            for (int64_t b = 0; b < jobs[i].nblocks; ++b) map[(size_t)(jobs[i].block0 + b)] = (uint32_t)i;
    }
    void *t = nullptr, *m = nullptr;
    if (hipMalloc(&t, sizeof(J) * jobs.size()) != hipSuccess) return KS_ENOMEM;
    allocs.push_back(t);
    if (hipMalloc(&m, sizeof(uint32_t) * std::max<int64_t>(nb, 1)) != hipSuccess) return KS_ENOMEM;
    allocs.push_back(m);
    if (hipMemcpy(t, jobs.data(), sizeof(J) * jobs.size(), hipMemcpyHostToDevice) != hipSuccess) return KS_EHIP;
    if (nb > 0 && hipMemcpy(m, map.data(), sizeof(uint32_t) * nb, hipMemcpyHostToDevice) != hipSuccess)
        return KS_EHIP;
    d.table = t;
    d.block_job = reinterpret_cast<uint32_t *>(m);
    return KS_OK;
}

// Lists keyed by digit width -> one list under key 0 (the launchers' "any width" kernel), the
// jobs' first blocks renumbered; a single width keeps its specialised kernel.
template <class J>
static void merge_widths(std::map<int, std::vector<J>> &lists) {
    if (lists.size() <= 1) return;
    std::vector<J> all;
    int64_t b = 0;
    for (auto &kv : lists)
        for (J j : kv.second) {
            j.block0 = b;
            b += j.nblocks;
            all.push_back(j);
        }
    lists.clear();
    lists[0] = std::move(all);
}

template <class J>
static int64_t blocks_of(const std::vector<J> &v) {
    return v.empty() ? 0 : v.back().block0 + v.back().nblocks;
}

}  // namespace ks

struct ks_batch_plan {
    int64_t count = 0;
    ks::JobLists JL;
    ks::DevTables T;
    std::vector<void *> allocs;
    int64_t status_words = 0;
    int64_t header_words = 0;  // status word, look-back words and ticket counters (cleared each run)
    int64_t ctr_pack = 0, ctr_norm = 0;  // word offsets of the counters
    int64_t ws_bytes = 0;
    double limb_mults = 0, school_mults = 0, hbm_bytes = 0;
    double pack_bytes = 0, normalize_bytes = 0, finish_bytes = 0, anchor_mults = 0, mfma_ops = 0, valu_mults = 0;
    double ntt_butterflies = 0;
    int32_t ntt_k1 = 0, ntt_k2 = 0;  // the first product on the transform engine
    int32_t engines = 0;  // OR of the engines the products use
    int variant = -1;
    // polynomial-level Karatsuba (every product modular, equal lengths, long): the three
    // half-length products of each product run as the batch plan `inner`, whose workspace
    // starts the workspace (its status word is this plan's); the staged halves and the three
    // sub-products follow at kara_in / kara_out bytes
    ks_batch_plan *inner = nullptr;
    ks::KaraProd *kara_tab = nullptr;  // device table, `count` entries
    int64_t kara_in = 0, kara_out = 0, kara_max_h = 0, kara_max_out = 0;
};

using namespace ks;

static const int64_t WS_DEVSTAT = 0, WS_STATUS = 64;

namespace ks {
// A run of a batch plan whose device status goes to `devstat` (a library-owned stream status
// word) instead of the workspace's own word: the bivariate products run their univariate
// products as one batch and report through the stream.
int batch_run_into(const ks_batch_plan *plan, const uint32_t *arena_in, uint32_t *arena_out, char *ws,
                   uint32_t *devstat, hipStream_t s) {
    if (plan->inner) {
        uint64_t *sub_in = reinterpret_cast<uint64_t *>(ws + plan->kara_in);
        uint64_t *sub_out = reinterpret_cast<uint64_t *>(ws + plan->kara_out);
        hipError_t e = timed_launch("kara", s, [&] {
            return launch_kara_split(plan->kara_tab, plan->count, plan->kara_max_h, arena_in, sub_in, s);
        });
        if (e != hipSuccess) return KS_EHIP;
        int rc = batch_run_into(plan->inner, reinterpret_cast<const uint32_t *>(sub_in),
                                reinterpret_cast<uint32_t *>(sub_out), ws, devstat, s);
        if (rc != KS_OK) return rc;
        e = timed_launch("kara", s, [&] {
            return launch_kara_combine(plan->kara_tab, plan->count, plan->kara_max_out, sub_out, arena_out, s);
        });
        return e == hipSuccess ? KS_OK : KS_EHIP;
    }
    if (launch_fill_zero(reinterpret_cast<uint64_t *>(ws), plan->header_words, s) != hipSuccess) return KS_EHIP;
    LaunchEnv env;
    env.status = reinterpret_cast<uint64_t *>(ws + WS_STATUS);
    env.ctr_pack = reinterpret_cast<uint64_t *>(ws) + plan->ctr_pack;
    env.ctr_norm = reinterpret_cast<uint64_t *>(ws) + plan->ctr_norm;
    env.devstat = devstat;
    env.base_in = reinterpret_cast<uintptr_t>(arena_in);
    env.base_out = reinterpret_cast<uintptr_t>(arena_out);
    env.base_ws = reinterpret_cast<uintptr_t>(ws);
    return launch_lists(plan->JL, &plan->T, env, 1u, 2u, s);
}
}  // namespace ks

extern "C" {

int64_t ks_batch_plan_bad_index(void) { return g_bad_index; }

void ks_batch_plan_destroy(ks_batch_plan *plan) {
    if (!plan) return;
    ks_batch_plan_destroy(plan->inner);
    for (void *p : plan->allocs) hipFree(p);
    delete plan;
}

static int plan_create(const ks_desc *descs, int64_t count, int32_t variant, bool allow_split,
                       ks_batch_plan **out);

int ks_batch_plan_create(const ks_desc *descs, int64_t count, int32_t variant, ks_batch_plan **out) {
    return plan_create(descs, count, variant, true, out);
}

// Every product modular (valid p, even offsets), both inputs of one length L >= 2, and the
// planner's integer operands (for the batch's variant) long enough: at least 8 t limbs over
// the batch (t = KS_KARATSUBA_MIN_LIMBS) and, in every product, t limbs, or 2 t once the batch
// holds 128 t.  Then the batch is split by one Karatsuba level, whose three half-length
// products are planned the same way, so the split recurses while they qualify.  Anything else
// is planned as it is (and an invalid descriptor is reported there).  A level saves a quarter
// of the multiplication and adds half again to the linear stages and two launches.  Measured
// (60-bit p): 64 products at L = 65536 paid down to operands of ~35K limbs -- four points 18.2
// ms unsplit, 15.3 / 14.3 / 15.3 ms with 1 / 2 / 3 levels, standard 71.2, 32.2 (2 levels),
// 22.9 (4), 25.0 ms (5) -- while the bivariate 16 x 4096 product's two or four products of
// 32K-64K terms paid down to ~17K limbs (four points 0.556 -> 0.487 ms, negated points
// 0.813 -> 0.598 ms) and lost with a single level.
static bool karatsuba_applies(const ks_desc *descs, int64_t count, int32_t variant) {
    const int64_t thr = env_int("KS_KARATSUBA_MIN_LIMBS", KARATSUBA_MIN_LIMBS);
    if (thr <= 0 || count > 65535) return false;
    int64_t total = 0, shortest = INT64_MAX;
    for (int64_t i = 0; i < count; ++i) {
        const ks_desc &d = descs[i];
        const uint64_t p = d.mod_p;
        if (d.flags != KS_MOD || p < 2 || (p >> 62) || (d.f_off & 1) || (d.g_off & 1) || (d.h_off & 1))
            return false;
        if (d.len_f != d.len_g || d.len_f < 2) return false;
        const int v = variant & KS_VARIANT_MASK;
        if (validate_spec(d.len_f, d.len_g, bitlen_u64(p - 1), v, true) != KS_OK) return false;
        Spec sp{d.len_f, d.len_g, bitlen_u64(p - 1), 2, false, p, v, variant & KS_ENGINE_ANY};
        sp.batch = true;
        sp.batch_count = count;
        sp.fill_blocks = std::max<int64_t>(1, 2048 / count);
        Geom G;
        if (plan_product(sp, G) != KS_OK) return false;
        // a quasi-linear product gains nothing from the split
        if (!G.muls.empty() && G.muls[0].engine == KS_ENGINE_NTT) return false;
        const int64_t n = std::min(G.nf, G.ng);
        if (n < thr) return false;
        shortest = std::min(shortest, n);
        total += n;
    }
    return total >= 8 * thr && shortest >= (total >= 128 * thr ? 2 * thr : thr);
}

}  // extern "C"

namespace ks {
bool karatsuba_splits(const ks_desc *descs, int64_t count, int32_t variant) {
    return karatsuba_applies(descs, count, variant);
}
}  // namespace ks

extern "C" {

static int plan_karatsuba(const ks_desc *descs, int64_t count, int32_t variant, ks_batch_plan **out) {
    std::vector<ks_desc> sub((size_t)(3 * count));
    std::vector<KaraProd> tab((size_t)count);
    int64_t nin = 0, nout = 0, max_h = 0, max_out = 0;
    double school = 0;
    for (int64_t i = 0; i < count; ++i) {
        const ks_desc &d = descs[i];
        KaraProd &K = tab[(size_t)i];
        K.f_off = d.f_off;
        K.g_off = d.g_off;
        K.h_off = d.h_off;
        K.L = d.len_f;
        K.h = (K.L + 1) / 2;
        K.p = d.mod_p;
        K.sub_in = nin;
        K.sub_out = nout;
        const int64_t m = 2 * K.h - 1;
        // f0 g0 -> z0, f1 g1 -> z2, (f0+f1)(g0+g1) -> z1 (residue offsets x 2 = uint32 words)
        const int64_t ins[3][2] = {{0, 3}, {1, 4}, {2, 5}};
        for (int t = 0; t < 3; ++t) {
            ks_desc &e = sub[(size_t)(3 * i + t)];
            memset(&e, 0, sizeof(e));
            e.f_off = (uint64_t)(2 * (nin + ins[t][0] * K.h));
            e.g_off = (uint64_t)(2 * (nin + ins[t][1] * K.h));
            e.h_off = (uint64_t)(2 * (nout + t * m));
            e.len_f = e.len_g = (int32_t)K.h;
            e.flags = KS_MOD;
            e.mod_p = d.mod_p;
        }
        nin += 6 * K.h;
        nout += 3 * m;
        max_h = std::max(max_h, K.h);
        max_out = std::max(max_out, 2 * K.L - 1);
        // the schoolbook count of the unsplit product, for the plan's totals
        Spec sp{d.len_f, d.len_g, bitlen_u64(d.mod_p - 1), 2, false, d.mod_p, variant & KS_VARIANT_MASK,
                variant & KS_ENGINE_ANY};
        sp.batch = true;
        sp.batch_count = count;
        sp.fill_blocks = std::max<int64_t>(1, 2048 / count);
        Geom G;
        if (plan_product(sp, G) == KS_OK) school += G.school_mults;
    }
    ks_batch_plan *inner = nullptr;
    int rc = plan_create(sub.data(), 3 * count, variant, true, &inner);
    if (rc != KS_OK) {
        g_bad_index = -1;  // the halves are not the caller's descriptors
        return rc;
    }
    ks_batch_plan *P = new ks_batch_plan();
    P->count = count;
    P->inner = inner;
    P->kara_in = align256(inner->ws_bytes);
    P->kara_out = align256(P->kara_in + 8 * nin);
    P->ws_bytes = align256(P->kara_out + 8 * nout);
    P->kara_max_h = max_h;
    P->kara_max_out = max_out;
    P->limb_mults = inner->limb_mults;
    P->school_mults = school;
    P->hbm_bytes = inner->hbm_bytes;
    P->pack_bytes = inner->pack_bytes;
    P->normalize_bytes = inner->normalize_bytes;
    P->finish_bytes = inner->finish_bytes;
    P->anchor_mults = inner->anchor_mults;
    P->mfma_ops = inner->mfma_ops;
    P->valu_mults = inner->valu_mults;
    P->ntt_butterflies = inner->ntt_butterflies;
    P->ntt_k1 = inner->ntt_k1;
    P->ntt_k2 = inner->ntt_k2;
    P->engines = inner->engines;
    P->variant = inner->variant;
    void *t = nullptr;
    if (hipMalloc(&t, sizeof(KaraProd) * tab.size()) != hipSuccess) { ks_batch_plan_destroy(P); return KS_ENOMEM; }
    P->allocs.push_back(t);
    if (hipMemcpy(t, tab.data(), sizeof(KaraProd) * tab.size(), hipMemcpyHostToDevice) != hipSuccess) {
        ks_batch_plan_destroy(P);
        return KS_EHIP;
    }
    P->kara_tab = reinterpret_cast<KaraProd *>(t);
    *out = P;
    return KS_OK;
}

static int plan_create(const ks_desc *descs, int64_t count, int32_t variant, bool allow_split,
                       ks_batch_plan **out) {
    g_bad_index = -1;
    if (!descs || !out || count < 1) return KS_EINVAL;
    *out = nullptr;
    const int known = KS_VARIANT_MASK | KS_SIGNED | KS_ENGINE_ANY;
    if (variant & ~known) return KS_EINVAL;
    const int v = variant & KS_VARIANT_MASK;
    const int eng = variant & KS_ENGINE_ANY;
    if (eng & (eng - 1)) return KS_EINVAL;  // at most one engine
    if (v != KS_VARIANT_AUTO && v != KS_VARIANT_KS1 && v != KS_VARIANT_NEG2 && v != KS_VARIANT_RECIP2 &&
        v != KS_VARIANT_KS4)
        return KS_EINVAL;
    if (allow_split && karatsuba_applies(descs, count, variant)) return plan_karatsuba(descs, count, variant, out);
    ks_batch_plan *P = new ks_batch_plan();
    P->count = count;
    int64_t off = align256(WS_STATUS);  // product scratch starts after the status words (fixed below)
    std::vector<Geom> geoms((size_t)count);
    std::vector<int64_t> inst_off((size_t)count);
    int64_t scratch = 0;
    for (int64_t i = 0; i < count; ++i) {
        const ks_desc &d = descs[i];
        Spec sp;
        const bool mod = (d.flags & KS_MOD) != 0;
        if (d.flags & ~(KS_SIGNED | KS_MOD)) { g_bad_index = i; delete P; return KS_EINVAL; }
        if (mod) {
            const uint64_t p = d.mod_p;
            if (p < 2 || (p >> 62) || (d.flags & KS_SIGNED) || (d.f_off & 1) || (d.g_off & 1) || (d.h_off & 1)) {
                g_bad_index = i;
                delete P;
                return KS_EINVAL;
            }
            sp = Spec{d.len_f, d.len_g, bitlen_u64(p - 1), 2, false, p, v, eng};
        } else {
            sp = Spec{d.len_f, d.len_g, d.coeff_bits, (d.coeff_bits + 31) / 32, (d.flags & KS_SIGNED) != 0, 0, v,
                      eng};
        }
        sp.batch = true;
        sp.batch_count = count;
        sp.fill_blocks = std::max<int64_t>(1, 2048 / count);
        if (validate_spec(sp.lf, sp.lg, sp.bits, v, true) != KS_OK) { g_bad_index = i; delete P; return KS_EINVAL; }
        int rc = plan_product(sp, geoms[(size_t)i]);
        if (rc != KS_OK) { g_bad_index = i; delete P; return rc; }
        inst_off[(size_t)i] = scratch;
        scratch += align256(geoms[(size_t)i].ws_status);  // the product's own scratch regions
        P->limb_mults += geoms[(size_t)i].limb_mults;
        P->school_mults += geoms[(size_t)i].school_mults;
        P->hbm_bytes += geoms[(size_t)i].hbm_bytes;
        P->pack_bytes += geoms[(size_t)i].pack_bytes;
        P->normalize_bytes += geoms[(size_t)i].normalize_bytes;
        P->finish_bytes += geoms[(size_t)i].finish_bytes;
        P->anchor_mults += geoms[(size_t)i].anchor_mults;
        P->mfma_ops += geoms[(size_t)i].mfma_ops;
        P->valu_mults += geoms[(size_t)i].valu_mults;
        P->ntt_butterflies += geoms[(size_t)i].ntt_butterflies;
        for (const auto &m : geoms[(size_t)i].muls)
            if (m.engine == KS_ENGINE_NTT && P->ntt_k1 == 0) {
                P->ntt_k1 = m.ntt_k1;
                P->ntt_k2 = m.ntt_k2;
            }
        for (const auto &m : geoms[(size_t)i].muls) P->engines |= m.engine;
        int rv = geoms[(size_t)i].variant;
        P->variant = i == 0 ? rv : (P->variant == rv ? rv : -1);
    }
    // jobs with offsets relative to the run's bases; scratch placed after the status words,
    // whose count is only known once every job is emitted -- emit relative to 0, then shift
    JobLists JL;
    for (int64_t i = 0; i < count; ++i) {
        const ks_desc &d = descs[i];
        emit_jobs(geoms[(size_t)i], (uintptr_t)(4 * d.f_off), (uintptr_t)(4 * d.g_off), (uintptr_t)(4 * d.h_off),
                  (uintptr_t)inst_off[(size_t)i], JL);
    }
    P->status_words = std::max(blocks_of(JL.pack), assign_dual_status(JL));
    P->ctr_pack = WS_STATUS / 8 + std::max<int64_t>(P->status_words, 1);
    P->ctr_norm = P->ctr_pack + (int64_t)JL.pack.size();
    P->header_words = P->ctr_norm + (int64_t)JL.norm.size();
    const int64_t base = align256(8 * P->header_words);
    auto sh = [&](auto *&ptr) { ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(reinterpret_cast<uintptr_t>(ptr) + base); };
    for (auto &j : JL.pack) sh(j.out);
    for (auto &j : JL.pack_small) sh(j.out);
    for (auto &j : JL.mul) { sh(j.a); sh(j.b); sh(j.cols); }
    for (auto &j : JL.mul_wave) { sh(j.a); sh(j.b); sh(j.cols); }
    for (auto &j : JL.digit) { sh(j.limbs); sh(j.out); sh(j.zero); }
    for (auto &j : JL.mfma) { sh(j.ad); sh(j.bd); sh(j.cols); }
    for (auto *nl : {&JL.ntt_f1, &JL.ntt_rows, &JL.ntt_i1})
        for (auto &j : *nl) {  // offsets (0 is a valid one); unused fields are never read
            sh(j.a);
            sh(j.x);
            sh(j.y);
        }
    for (auto &j : JL.ntt_join) {
        sh(j.x);
        sh(j.cols);
    }
    for (auto &kv : JL.anchor) for (auto &j : kv.second) { sh(j.anchors); sh(j.anchors2); }
    for (auto *nl : {&JL.norm, &JL.norm_small})
        for (auto &j : *nl) {
            for (int q = 0; q < j.nterms; ++q) { sh(j.term[q].cols); sh(j.term[q].a); sh(j.term[q].b); }
            sh(j.out);
            sh(j.out2);
        }
    for (auto &j : JL.extract) sh(j.src);
    for (auto &kv : JL.chain) for (auto &j : kv.second) { sh(j.A); sh(j.B); sh(j.anchors); sh(j.hbuf); }
    for (auto &kv : JL.finish) for (auto &j : kv.second) { sh(j.A); sh(j.B); sh(j.anchors); sh(j.hbuf); }
    P->ws_bytes = base + scratch;
    (void)off;
    // a batch's chains are launched by segment (one lane each, jobs packed side by side in the
    // waves), and chains (and finishing passes) of several digit widths go into one launch
    // whose lanes (blocks) run their own width, rather than one launch per width in turn
    for (auto &kv : JL.chain) {
        int64_t b = 0;
        for (auto &j : kv.second) {
            j.block0 = b;
            j.nblocks = j.nseg;
            b += j.nseg;
        }
    }
    merge_widths(JL.chain);
    merge_widths(JL.finish);

    int rc = KS_OK;
    if (!JL.ntt_f1.empty()) rc = ntt_prepare();  // the transforms' root tables on this device
    if (rc == KS_OK) rc = upload(JL.pack, P->T.pack, P->allocs, true);
    if (rc == KS_OK) rc = upload(JL.ntt_f1, P->T.ntt_f1, P->allocs);
    if (rc == KS_OK) rc = upload(JL.ntt_rows, P->T.ntt_rows, P->allocs);
    if (rc == KS_OK) rc = upload(JL.ntt_i1, P->T.ntt_i1, P->allocs);
    if (rc == KS_OK) rc = upload(JL.ntt_join, P->T.ntt_join, P->allocs);
    if (rc == KS_OK) rc = upload(JL.pack_small, P->T.pack_small, P->allocs, true);
    if (rc == KS_OK) rc = upload(JL.mul, P->T.mul, P->allocs);
    if (rc == KS_OK) rc = upload(JL.mul_wave, P->T.mul_wave, P->allocs);
    if (rc == KS_OK) rc = upload(JL.digit, P->T.digit, P->allocs);
    if (rc == KS_OK) rc = upload(JL.mfma, P->T.mfma, P->allocs);
    if (rc == KS_OK) rc = upload(JL.norm, P->T.norm, P->allocs, true);
    if (rc == KS_OK) rc = upload(JL.norm_small, P->T.norm_small, P->allocs, true);
    if (rc == KS_OK) rc = upload(JL.extract, P->T.extract, P->allocs);
    for (auto &kv : JL.anchor) if (rc == KS_OK) rc = upload(kv.second, P->T.anchor[kv.first], P->allocs);
    for (auto &kv : JL.chain) if (rc == KS_OK) rc = upload(kv.second, P->T.chain[kv.first], P->allocs);
    for (auto &kv : JL.finish) if (rc == KS_OK) rc = upload(kv.second, P->T.finish[kv.first], P->allocs);
    if (rc != KS_OK) { ks_batch_plan_destroy(P); return rc; }
    P->JL = std::move(JL);
    *out = P;
    return KS_OK;
}

size_t ks_batch_plan_workspace_bytes(const ks_batch_plan *plan) { return plan ? (size_t)plan->ws_bytes : 0; }

int ks_batch_plan_info(const ks_batch_plan *plan, ks_plan_info *out) {
    if (!plan || !out) return KS_EINVAL;
    memset(out, 0, sizeof(*out));
    out->variant = plan->variant;
    out->engine = plan->engines ? plan->engines : KS_ENGINE_VALU;
    out->n_products = (int32_t)std::min<int64_t>(plan->count, 0x7fffffff);
    out->limb_mults = plan->limb_mults;
    out->schoolbook_limb_mults = plan->school_mults;
    out->hbm_bytes = plan->hbm_bytes;
    out->pack_bytes = plan->pack_bytes;
    out->normalize_bytes = plan->normalize_bytes;
    out->finish_bytes = plan->finish_bytes;
    out->anchor_limb_mults = plan->anchor_mults;
    out->mfma_ops = plan->mfma_ops;
    out->valu_limb_mults = plan->valu_mults;
    out->scratch_bytes = plan->ws_bytes;
    out->ntt_butterflies = plan->ntt_butterflies;
    out->ntt_k1 = plan->ntt_k1;
    out->ntt_k2 = plan->ntt_k2;
    return KS_OK;
}

int ks_batch_run(const ks_batch_plan *plan, const uint32_t *arena_in, uint32_t *arena_out, void *workspace,
                 size_t ws_bytes, void *stream) {
    if (!plan || !arena_in || !arena_out || !workspace) return KS_EINVAL;
    if (ws_bytes < (size_t)plan->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255)) return KS_EINVAL;
    if (device_ok() != 1) return KS_EUNSUPPORTED;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    // the status word, ticket counters and look-back words start every run at zero (a kernel,
    // not a memset, so the run can be graph-captured); the status thus reports the latest run
    return batch_run_into(plan, arena_in, arena_out, ws, reinterpret_cast<uint32_t *>(ws + WS_DEVSTAT), s);
}

int ks_batch_status(const ks_batch_plan *plan, void *workspace, void *stream) {
    if (!plan || !workspace) return KS_EINVAL;
    return read_status(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(workspace) + WS_DEVSTAT),
                       reinterpret_cast<hipStream_t>(stream));
}

size_t ks_batch_workspace_bytes(const ks_desc *descs, int64_t count, int32_t variant) {
    ks_batch_plan *P = nullptr;
    if (ks_batch_plan_create(descs, count, variant, &P) != KS_OK) return 0;
    size_t b = (size_t)P->ws_bytes;
    ks_batch_plan_destroy(P);
    return b;
}

int ks_mul_batch(const uint32_t *arena_in, uint32_t *arena_out, const ks_desc *descs, int64_t count, int32_t variant,
                 void *workspace, size_t ws_bytes, void *stream) {
    ks_batch_plan *P = nullptr;
    int rc = ks_batch_plan_create(descs, count, variant, &P);
    if (rc != KS_OK) return rc;
    rc = ks_batch_run(P, arena_in, arena_out, workspace, ws_bytes, stream);
    // the plan's tables must outlive the kernels that read them
    if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess && rc == KS_OK) rc = KS_EHIP;
    ks_batch_plan_destroy(P);
    return rc;
}

}  // extern "C"
