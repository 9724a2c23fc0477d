// ks_api.cpp -- host side of libksmul: planner, scratch pools, launch sequencing, C ABI.
//
// One product runs as a short pipeline of kernels on the caller's stream:
//   pack       evaluations of f and g at the variant's points        (paper 3.1, 3.3, 3.4)
//   mul_valu   the 1, 2 or 4 integer products                        (3.1 - 3.4)
//   normalize  carry resolution, recombination and exact halving     (3.3, 3.4)
//   extract    coefficients read off their slots                     (3.1, 3.3)
//   anchor + chain   Section 3.2's reconstruction, in parallel segments  (3.4)
// The planner below turns (lengths, bits, variant) into sizes and job descriptors; the same
// descriptors drive single products (passed by value) and batches (device tables).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ks.h"
#include "ks_jobs.h"
#include "ks_launch.h"
#include "ks_plan.h"

namespace ks {

// ---- small integer helpers --------------------------------------------------------------------

int ceil_log2(int64_t x) {
    int e = 0;
    while (((int64_t)1 << e) < x) ++e;
    return e;
}
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t align_up(int64_t x, int64_t a) { return cdiv(x, a) * a; }

// planner tunables: a value set through ks_tune_set, else the environment, else the default
static const char *const k_tunables[] = {"KS_MFMA_MIN_LIMBS", "KS_MFMA_BLOCKS",  "KS_MFMA_MIN_PART",
                                         "KS_MFMA_BLOCK_COST", "KS_CHAIN_K",     "KS_MUL_WAVE_MAX",
                                         "KS_SCAN_SMALL",      "KS_MFMA_RT",      "KS_KARATSUBA_MIN_LIMBS",
                                         "KS_NTT_MIN_LIMBS",   "KS_SCAN_BIG"};
static std::mutex g_tune_mu;
static std::map<std::string, int64_t> g_tune;
static uint64_t g_tune_gen = 0;  // bumped by every ks_tune_set / ks_tune_reset

uint64_t tune_generation() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune_gen;
}

static bool known_tunable(const char *name) {
    for (const char *k : k_tunables)
        if (strcmp(k, name) == 0) return true;
    return false;
}

// Tunables from the autotuner's JSON cache, read once per process: the file KS_TUNING_FILE
// names, else $XDG_CACHE_HOME/ksmul/tuning.json or $HOME/.cache/ksmul/tuning.json when present.
// Every `"NAME": integer` pair of a known tunable in it is taken (the autotuner writes them under
// "tunables"); anything else in the file is ignored.
static const std::map<std::string, int64_t> &file_tunables() {
    static std::map<std::string, int64_t> table;
    static std::once_flag once;
    std::call_once(once, [] {
        std::string path;
        if (const char *f = getenv("KS_TUNING_FILE")) path = f;
        else if (const char *x = getenv("XDG_CACHE_HOME")) path = std::string(x) + "/ksmul/tuning.json";
        else if (const char *h = getenv("HOME")) path = std::string(h) + "/.cache/ksmul/tuning.json";
        if (path.empty()) return;
        FILE *fh = fopen(path.c_str(), "rb");
        if (!fh) return;
        std::string txt;
        char buf[4096];
        size_t n;
        while ((n = fread(buf, 1, sizeof(buf), fh)) > 0 && txt.size() < (1u << 20)) txt.append(buf, n);
        fclose(fh);
        for (const char *k : k_tunables) {
            const std::string key = std::string("\"") + k + "\"";
            const size_t at = txt.find(key);
            if (at == std::string::npos) continue;
            size_t i = at + key.size();
            while (i < txt.size() && (txt[i] == ' ' || txt[i] == '\t' || txt[i] == '\n' || txt[i] == '\r')) ++i;
            if (i >= txt.size() || txt[i] != ':') continue;
            char *end = nullptr;
            const long long v = strtoll(txt.c_str() + i + 1, &end, 10);
            if (end != txt.c_str() + i + 1 && v >= 0) table[k] = v;
        }
    });
    return table;
}

int env_int(const char *name, int dflt) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(name);
        if (it != g_tune.end()) return (int)std::min<int64_t>(it->second, 0x7fffffff);
    }
    const char *v = getenv(name);
    if (v && *v) return atoi(v);
    const auto &ft = file_tunables();
    auto it = ft.find(name);
    return it != ft.end() ? (int)std::min<int64_t>(it->second, 0x7fffffff) : dflt;
}

// ---- planning -----------------------------------------------------------------------------------

// Launch shape of the matrix-core products: parts per row group (splits) and residue groups
// per part (rgroups) for `units` row groups of at most tmax block shifts each.  Every block
// covers at least min_part shifts (unless one part per residue group is already shorter).
// target > 0: aim at about `target` blocks, cutting the residues first (a wave's shifts then
// form fewer, longer chains) and the shift range after.  target = 0: the shape of least
// modelled time, the blocks running one per compute unit in rounds of MFMA_CUS, each taking
// a fixed cost (start, LDS and column sums: KS_MFMA_BLOCK_COST steps), the start-up of each
// residue class of a wave (its first loads: about MFMA_CLASS_COST steps) and its steps (a
// step: MFMA_RT matrix operations of each wave).
static constexpr int64_t MFMA_CUS = 256, MFMA_CLASS_COST = 3;
// a single product whose launch has at most this many 8-tile row groups uses 4-tile blocks
static constexpr int64_t MFMA_RT4_MAX_GROUPS = 256;
static void mfma_shape(int64_t tmax, int64_t units, int64_t target, int64_t min_part, int64_t &splits,
                       int64_t &rgroups) {
    min_part = std::max<int64_t>(1, min_part);
    auto s_min = [&](int64_t rg) { return cdiv(tmax, mfma_max_part(rg)); };
    if (target > 0) {
        const int64_t d = cdiv(target, units);
        rgroups = d >= 4 ? 4 : d >= 2 ? 2 : 1;
        const int64_t s_cap = std::max<int64_t>(1, tmax / (rgroups * min_part));
        splits = std::max(s_min(rgroups), std::min(cdiv(d, rgroups), s_cap));
        return;
    }
    const int64_t c0 = env_int("KS_MFMA_BLOCK_COST", 10);
    double best = 0;
    splits = s_min(1);
    rgroups = 1;
    for (int64_t rg = 1; rg <= 4; rg *= 2) {
        const int64_t cpw = MFMA_CLASSES / rg;
        for (int64_t s = s_min(rg); s <= std::max(s_min(rg), cdiv(4 * MFMA_CUS, units * rg)); ++s) {
            const int64_t part = cdiv(tmax, s);
            const int64_t steps = cpw * cdiv(part, 32);  // per wave
            if (s > s_min(rg) && part < rg * min_part) break;
            const double t = (double)cdiv(units * rg * s, MFMA_CUS) * (double)(c0 + cpw * MFMA_CLASS_COST + steps);
            if (best == 0 || t < best) {
                best = t;
                splits = s;
                rgroups = rg;
            }
        }
    }
}

static int64_t slot_bits(int variant, int b, int e) {
    switch (variant) {
        case KS_VARIANT_KS1: return 2 * (int64_t)b + e;                 // Section 3.1
        case KS_VARIANT_NEG2: return (int64_t)b + (e + 1) / 2;          // Section 3.3
        case KS_VARIANT_RECIP2: return (int64_t)b + (e + 1) / 2;        // Section 3.2
        case KS_VARIANT_KS4: return (2 * (int64_t)b + e + 3) / 4;       // Section 3.4
    }
    return 0;
}

// Time model for KS_VARIANT_AUTO (microseconds on one MI355X, fitted to single-product
// measurements): the products on the engine the planner will pick -- vector ALU 0.21 fs per
// limb product above a 5 us floor, matrix cores 0.69 fs per int8 operation on balanced digits
// above a 10 us floor, transforms 3.5 ps per term and level -- plus 0.15 ns per operand limb
// for the linear stages, 0.2 ns per coefficient for KS4's reconstruction, and 4.5 us per launch
// (KS4 has one more; the matrix cores add the digit launch, the transforms four).  A batch
// shares its launches, so there only the rates count.  With the quasi-linear transforms the
// four products of a quarter of the length cost about as much as the one long product, and the
// standard substitution's lighter linear stages win (Section 1: the gain of several points
// vanishes as M(b) approaches b log b).
// It picks NEG2 for the L = 4096 signed 64-bit product (measured 0.043 ms, against 0.045 for
// KS1 and 0.051 for KS4), KS4 for L = 65536 at 48 bits (0.54 ms, against 0.72 and 1.27), and
// KS1 or NEG2 for short products, where every variant is launch-bound.
static int auto_variant(int64_t lf, int64_t lg, int b, int e, bool batch, int engine) {
    double best = 1e300;
    int pick = KS_VARIANT_KS1;
    for (int v : {KS_VARIANT_KS1, KS_VARIANT_NEG2, KS_VARIANT_KS4}) {
        const int64_t N = slot_bits(v, b, e);
        const int k = v == KS_VARIANT_KS1 ? 1 : (v == KS_VARIANT_NEG2 ? 2 : 4);
        const double na = (double)cdiv(N * (lf - 1) + b + 2, 32), nb = (double)cdiv(N * (lg - 1) + b + 2, 32);
        int eng = engine;
        int k1 = 0, k2 = 0, w = 0;
        int64_t pa = 0, pb = 0;
        const bool ntt_ok = ntt_shape((int64_t)na, (int64_t)nb, 0, k1, k2, w, pa, pb);
        const int64_t ntt_min = env_int("KS_NTT_MIN_LIMBS", batch ? NTT_MIN_LIMBS_BATCH : NTT_MIN_LIMBS);
        if (eng == 0 && ntt_ok && ntt_min > 0 && std::min(na, nb) >= (double)ntt_min) eng = KS_ENGINE_NTT;
        if (eng == KS_ENGINE_NTT && !ntt_ok) eng = KS_ENGINE_MFMA;
        if (eng == 0)
            eng = std::min(na, nb) >= env_int("KS_MFMA_MIN_LIMBS", batch ? 1000 : 2500) ? KS_ENGINE_MFMA : KS_ENGINE_VALU;
        double us = 0;
        int launches = 4;  // pack, multiply, recombine, extract
        if (eng == KS_ENGINE_NTT) {
            // 3.5 ps per transform term and level (both primes, three transforms and the join;
            // 0.34 ms for one product through 2^22 terms, 3.9 ms for 256 through 2^18)
            us += k * 3.5e-6 * (double)((int64_t)1 << (k1 + k2)) * (k1 + k2);
            launches += 4;  // four transform steps and the join in place of one multiplier
        } else if (eng == KS_ENGINE_MFMA) {
            us += k * 2.0 * (4 * na + 1) * (4 * nb + 1) * 6.9e-10;
            launches += 1;  // digits
            if (!batch) us += 10.0;
        } else {
            us += k * na * nb * 2.1e-7;
            if (!batch) us += 5.0;
        }
        if (v == KS_VARIANT_KS4) {
            launches += 1;  // reconstruction chain and its finishing pass in place of extraction
            us += 2e-4 * (double)(lf + lg);
        }
        us += 1.5e-4 * k * (na + nb);
        if (!batch) us += 4.5 * launches;
        if (us < best) { best = us; pick = v; }
    }
    return pick;
}

int plan_product(const Spec &sp, Geom &G) {
    G = Geom();
    G.sp = sp;
    G.ipt = sp.batch ? SCAN_IPT_BATCH : SCAN_IPT_SINGLE;
    G.pack_ipt = sp.batch ? PACK_IPT_BATCH : SCAN_IPT_SINGLE;
    const int64_t lf = sp.lf, lg = sp.lg;
    const int b = sp.bits;
    G.e = ceil_log2(std::min(lf, lg));
    G.D = lf + lg - 1;
    G.m0 = (G.D + 1) / 2;
    G.m1 = G.D / 2;
    G.w_out = (int)cdiv(2 * (int64_t)b + G.e + 1, 32);
    G.off = sp.sgn ? 2 * b - 2 + G.e : -1;
    int v = sp.variant;
    if (v == KS_VARIANT_AUTO) v = auto_variant(lf, lg, b, G.e, sp.batch, sp.engine);
    if (v != KS_VARIANT_KS1 && v != KS_VARIANT_NEG2 && v != KS_VARIANT_RECIP2 && v != KS_VARIANT_KS4)
        return KS_EINVAL;
    G.variant = v;
    const int64_t N = slot_bits(v, b, G.e);
    G.N = N;
    const int64_t nf = cdiv(N * (lf - 1) + b + 2, 32), ng = cdiv(N * (lg - 1) + b + 2, 32);
    G.nf = nf;
    G.ng = ng;
    // A single product whose result holds many limbs is bound by throughput like a batch: it
    // takes a batch's carry-scan blocks, which pay the ticket and the look-back over twice or
    // four times as many limbs (L = 65536, b = 256: 0.35 -> 0.29 ms standard, 0.70 -> 0.57 ms
    // four-point).  Small ones keep the short blocks that their latency favours.
    const int64_t big_min = env_int("KS_SCAN_BIG", SCAN_BIG_LIMBS);
    if (!sp.batch && big_min > 0 && G.D * (2 * (int64_t)b + G.e) / 32 >= big_min) {
        G.ipt = SCAN_IPT_BATCH;
        G.pack_ipt = PACK_IPT_BATCH;
    }

    // evaluations: f points first, then the same points for g
    std::vector<int> pf;
    if (v == KS_VARIANT_KS1) pf = {0};
    else if (v == KS_VARIANT_NEG2) pf = {0, PK_ALTERNATE};
    else if (v == KS_VARIANT_RECIP2) pf = {0, PK_REVERSE};
    else pf = {0, PK_ALTERNATE, PK_REVERSE, PK_REVERSE | PK_ALTERNATE};
    const int npts = (int)pf.size();
    int64_t off = 0;
    for (int which = 0; which < 2; ++which)
        for (int q = 0; q < npts; ++q) {
            PackGeom p;
            p.which = which;
            p.flags = pf[q] | (sp.sgn ? PK_SIGNED : 0) | (q == 0 ? PK_CHECK : 0);
            p.L = which ? lg : lf;
            p.n_out = which ? ng : nf;
            p.op_off = off;
            p.small = p.n_out <= std::min<int64_t>(small_bl(G.pack_ipt), env_int("KS_SCAN_SMALL", (int)small_bl(G.pack_ipt)));
            p.blocks = p.small ? 1 : cdiv(p.n_out, scan_bl(G.pack_ipt));
            off += align_up(p.n_out, 64);
            G.packs.push_back(p);
            G.pack_blocks += p.blocks;
        }
    G.op_limbs = off;

    // products: point q of f times point q of g, on the vector ALU or the matrix cores
    int64_t coff = 0, doff = 0;
    for (int q = 0; q < npts; ++q) {
        MulGeom m;
        m.fa = q;
        m.fb = npts + q;
        m.na = nf;
        m.nb = ng;
        m.nad = 4 * nf + 1;  // balanced 8-bit digits: one per byte and the top carry
        m.nbd = 4 * ng + 1;
        m.nA32 = cdiv(m.nad, 32);
        m.nB32 = cdiv(m.nbd + 31, 32);
        int eng = sp.engine;
        // long operands go through the transforms (quasi-linear), when a transform length fits
        const int64_t ntt_min = env_int("KS_NTT_MIN_LIMBS", sp.batch ? NTT_MIN_LIMBS_BATCH : NTT_MIN_LIMBS);
        if (eng == 0 && ntt_min > 0 && std::min(nf, ng) >= ntt_min &&
            ntt_shape(nf, ng, 0, m.ntt_k1, m.ntt_k2, m.ntt_w, m.ntt_npa, m.ntt_npb))
            eng = KS_ENGINE_NTT;
        if (eng == KS_ENGINE_NTT && !ntt_shape(nf, ng, 0, m.ntt_k1, m.ntt_k2, m.ntt_w, m.ntt_npa, m.ntt_npb))
            eng = KS_ENGINE_MFMA;  // beyond the longest transform
        // the matrix cores cost a digit launch more: a single product needs operands of about
        // 2200-2400 limbs to gain (vector ALU / matrix cores 0.99-1.01 there, 1.12-1.17 at
        // ~4400 limbs); a batch shares that launch among its products (10,000-product batch:
        // standard KS 1.95 ms at 2500 limbs, 1.77-1.81 ms at 800-1200; four-point 2.02 and
        // 1.91 ms)
        if (eng == 0)
            eng = std::min(nf, ng) >= env_int("KS_MFMA_MIN_LIMBS", sp.batch ? 1000 : 2500) ? KS_ENGINE_MFMA
                                                                                          : KS_ENGINE_VALU;
        m.engine = eng;
        if (eng == KS_ENGINE_NTT) {
            const int64_t Nt = (int64_t)1 << (m.ntt_k1 + m.ntt_k2);
            m.ntt_nz = m.ntt_npa + m.ntt_npb - 1;
            m.ntt_xa = G.ntt_words;
            m.ntt_xb = m.ntt_xa + 2 * Nt;
            m.ntt_cols = m.ntt_xb + 2 * Nt;
            m.ncols = m.ntt_w * (m.ntt_nz - 1) / 32 + 1;  // the last term's column
            G.ntt_words = m.ntt_cols + align_up(3 * m.ncols, 64);
            m.cols_off = -1;
            G.muls.push_back(m);
            G.school_mults += (double)nf * (double)ng;
            G.ntt_butterflies += 6.0 * (double)(Nt / 2) * (double)(m.ntt_k1 + m.ntt_k2);
            continue;
        }
        if (eng == KS_ENGINE_MFMA) {
            const int64_t rows = cdiv(m.nad + m.nbd - 1, 32);
            // row tiles per block: 8 share each loaded a-fragment among more matrix operations
            // (large products, batches); 4 give a small single product twice the blocks
            m.rt = env_int("KS_MFMA_RT", 0);
            if (m.rt != 4 && m.rt != 8)
                m.rt = (!sp.batch && (int64_t)npts * cdiv(rows, mfma_rows(8)) <= MFMA_RT4_MAX_GROUPS) ? 4 : 8;
            const int64_t grows = mfma_rows(m.rt), glimbs = mfma_limbs(m.rt);  // output rows, limbs of a group
            m.groups = cdiv(rows, grows);
            // the longest shift range of a row group, cut into parts of at most
            // mfma_max_part(rgroups) shifts (int32 accumulators), each shared by rgroups
            // blocks (residue groups)
            const int64_t tmax = std::min(m.nA32 + grows - 1, m.nB32);
            mfma_shape(tmax, (int64_t)npts * m.groups, env_int("KS_MFMA_BLOCKS", (int)sp.fill_blocks),
                       env_int("KS_MFMA_MIN_PART", 128), m.splits, m.rgroups);
            m.part = cdiv(tmax, m.splits);
            m.blocks = m.groups * m.splits * m.rgroups;
            m.ncols = m.groups * glimbs;
            m.a_front = 32 * grows;
            m.a_len = align_up(m.a_front + 32 * m.nA32 + 32 * grows, 1024);
            m.b_len = align_up(32 * m.nB32 + 2 * MFMA_PADB + 32, 1024);
            m.b_top = m.b_len - 1 - MFMA_PADB;
            m.ad_off = doff;
            doff += m.a_len;
            m.bd_off = doff;
            doff += m.b_len;
        } else {
            m.ntiles = cdiv(nf + ng - 1, MUL_T);
            m.blocks = m.ntiles;
            m.ncols = m.ntiles * MUL_T;
            // a tile's i range is at most min(nf, ng) limbs: when that is short, one wave per
            // tile keeps the waves busy (the block mode splits the range over MUL_WAVES waves)
            m.wave = std::min(nf, ng) <= env_int("KS_MUL_WAVE_MAX", sp.batch ? 1024 : 128);
        }
        m.cols_off = coff;
        coff += align_up((eng == KS_ENGINE_MFMA ? 4 : 3) * m.ncols, 64);
        G.muls.push_back(m);
        G.mul_blocks += m.blocks;
        G.school_mults += (double)nf * (double)ng;
        if (eng == KS_ENGINE_MFMA) G.mfma_ops += 2.0 * (double)m.nad * (double)m.nbd;
        else G.valu_mults += (double)nf * (double)ng;
    }
    G.col_words = coff;
    G.digit_bytes = doff;
    G.limb_mults = G.school_mults;

    // recombinations
    int64_t noff = 0;
    const int64_t prod_limbs = nf + ng;
    auto add_norm = [&](std::vector<int> prods, std::vector<int> signs, int64_t shift, int64_t obit, int64_t period,
                        int64_t count, int64_t n_out) {
        NormGeom r;
        r.nterms = (int)prods.size();
        for (int t = 0; t < r.nterms; ++t) { r.prod[t] = prods[t]; r.sign[t] = signs[t]; }
        r.shift = (int)shift;
        r.off_bit0 = obit;
        r.off_period = period;
        r.off_count = sp.sgn ? count : 0;
        r.n_out = n_out;
        r.n_in = std::max(prod_limbs + 2, n_out + shift / 32 + 2);
        r.small = r.n_in <= std::min<int64_t>(small_bl(G.ipt), env_int("KS_SCAN_SMALL", (int)small_bl(G.ipt)));
        r.blocks = r.small ? 1 : cdiv(r.n_in, scan_bl(G.ipt));
        r.out_off = noff;
        noff += align_up(n_out, 64);
        G.norms.push_back(r);
        G.norm_blocks += r.blocks;
        return (int)G.norms.size() - 1;
    };
    // Section 3.2's reconstruction of m coefficients from A = norm a (digits u, base 2^Nd) and
    // B = norm bb (digits w from the top); output coefficients first, first + step, ...
    // segment length K: every segment but the first costs one anchor (a dot product of
    // min(lf, lg) coefficient products, spread over the GPU), and a segment's lane runs K
    // dependent steps; K ~ sqrt(D L W^2 / c) balances the two (c from measurement: K = 8 is
    // the optimum of the L = 4096 product).  In a batch of n products the anchors of all
    // products share the GPU while their chains run side by side, which favours longer
    // segments: the factor sqrt(n), c = 2.8e5 and the floor of 384 match the measured optima of
    // the 10,000-product (K = 384: 1.39-1.40 ms against 1.41 at 256, 1.41-1.42 at 512 and 1.43
    // at 192) and 64-product modular workloads (K ~ 990: 2.31-2.35 ms at K = 900-1100 against
    // 2.40-2.45 at 741), with ~34 instructions a chain step and 16 steps in flight.
    auto add_chain = [&](int a, int bb, int64_t m, int first, int64_t Nd, int step) {
        const double Lm = (double)std::min(lf, lg);
        const double nbat = std::sqrt((double)sp.batch_count);
        const double cK = sp.batch ? 2.8e5 : 2.0e6;
        int64_t K = (int64_t)(std::sqrt(nbat * G.D * Lm * sp.w_in * sp.w_in / cK) + 0.5);
        K = std::max<int64_t>(sp.batch ? 384 : 4, std::min<int64_t>(K, 4096));
        const int64_t Kset = env_int("KS_CHAIN_K", 0);
        if (Kset > 0) K = Kset;
        G.nw = (int)cdiv(Nd, 32);
        G.chain_nd = Nd;
        G.aw = 2 * sp.w_in + 2;
        ChainGeom c;
        c.A = a;
        c.B = bb;
        c.m = m;
        c.K = K;
        c.nseg = cdiv(m, K);
        c.par = first;
        c.step = step;
        c.anchor_off = G.anchor_limbs;
        c.anchor_blocks = c.nseg - 1;
        c.chain_blocks = cdiv(c.nseg, CHAIN_TPB);
        c.hbuf_off = G.hbuf_words;
        c.finish_blocks = cdiv(m, FINISH_TPB);
        G.hbuf_words += align_up(m * 2 * cdiv(Nd, 32), 64);
        G.finish_blocks += c.finish_blocks;
        G.anchor_limbs += align_up(c.nseg * G.aw, 64);
        G.chains.push_back(c);
        G.anchor_blocks += c.anchor_blocks;
        G.chain_blocks += c.chain_blocks;
        G.anchor_mults += (double)(c.nseg - 1) * std::min(lf, lg) * sp.w_in * sp.w_in;
    };
    if (v == KS_VARIANT_KS1) {
        add_norm({0}, {1}, 0, G.off, N, G.D, cdiv(G.D * N, 32) + 1);
        ExtractGeom x{0, G.D, N, 0, 1, cdiv(G.D, EXTRACT_TPB)};
        G.extracts.push_back(x);
    } else if (v == KS_VARIANT_RECIP2) {
        // A = h(2^N) and B = h^rev(2^N) (Section 3.2), each with the slot constant, then the
        // reconstruction at base 2^N over all D coefficients
        const int64_t n_out = cdiv((G.D + 1) * N, 32) + 1;
        const int a = add_norm({0}, {1}, 0, G.off, N, G.D, n_out);
        const int bb = add_norm({1}, {1}, 0, G.off, N, G.D, n_out);
        add_chain(a, bb, G.D, 0, N, 1);
    } else {
        const int64_t Y = 2 * N;  // bits of the even/odd base 2^(2N)
        // P0 = (H1 + H2 + 2 C 1(Y)) / 2,  P1 = (H1 - H2 + 2^(N+1) C 1(Y)) / 2^(N+1)
        int p0 = add_norm({0, 1}, {1, 1}, 1, G.off + 1, Y, G.m0, cdiv((G.m0 + 1) * Y, 32) + 1);
        int p1 = -1;
        if (G.m1 > 0) p1 = add_norm({0, 1}, {1, -1}, N + 1, G.off + N + 1, Y, G.m1, cdiv((G.m1 + 1) * Y, 32) + 1);
        if (v == KS_VARIANT_NEG2) {
            G.extracts.push_back(ExtractGeom{p0, G.m0, Y, 0, 2, cdiv(G.m0, EXTRACT_TPB)});
            if (p1 >= 0) G.extracts.push_back(ExtractGeom{p1, G.m1, Y, 1, 2, cdiv(G.m1, EXTRACT_TPB)});
        } else {
            // reversed products: Q0 = even part of h^rev (m0 coefficients), Q1 = odd part (m1)
            int q0 = add_norm({2, 3}, {1, 1}, 1, G.off + 1, Y, G.m0, cdiv((G.m0 + 1) * Y, 32) + 1);
            int q1 = -1;
            if (G.m1 > 0) q1 = add_norm({2, 3}, {1, -1}, N + 1, G.off + N + 1, Y, G.m1, cdiv((G.m1 + 1) * Y, 32) + 1);
            const bool dodd = (G.D & 1) != 0;  // reversal swaps parities when D is even
            add_chain(p0, dodd ? q0 : q1, G.m0, 0, 2 * N, 2);
            if (G.m1 > 0) add_chain(p1, dodd ? q1 : q0, G.m1, 1, 2 * N, 2);
        }
    }
    G.norm_limbs = noff;
    // recombinations of the same two products with signs (+, +) and (+, -) -- P0 and P1, Q0 and
    // Q1 of the negated and four-point substitutions -- run as one job: the column windows are
    // read once and feed two carry scans (the second looks back through words of its own).  In
    // batches only: a single product is bound by latency, which the longer blocks raise (the
    // L = 4096 product's recombination 13 -> 18 us).
    for (size_t i = 0; sp.batch && i + 1 < G.norms.size(); ++i) {
        NormGeom &a = G.norms[i], &b = G.norms[i + 1];
        if (a.merged || a.small || b.small || a.nterms != 2 || b.nterms != 2 || a.prod[0] != b.prod[0] ||
            a.prod[1] != b.prod[1] || a.off_period != b.off_period || a.blocks != b.blocks)
            continue;
        a.pair = (int)(i + 1);
        b.merged = true;
        G.norm_status_extra += a.blocks;
    }
    for (auto &x : G.extracts) G.extract_blocks += x.blocks;

    // scratch layout (bytes)
    int64_t o = 0;
    G.ws_ops = o;     o += align_up(G.op_limbs * 4, 256);
    G.ws_cols = o;    o += align_up(G.col_words * 4, 256);
    G.ws_digits = o;  o += align_up(G.digit_bytes, 256);
    G.ws_norms = o;   o += align_up(G.norm_limbs * 4, 256);
    G.ws_anchors = o; o += align_up(std::max<int64_t>(G.anchor_limbs, 1) * 4, 256);
    G.ws_hbuf = o;    o += align_up(G.hbuf_words * 4, 256);
    G.ws_ntt = o;     o += align_up(G.ntt_words * 4, 256);
    G.ws_status = o;
    o += align_up(std::max<int64_t>(std::max(G.pack_blocks, G.norm_blocks + G.norm_status_extra), 1) * 8, 256);
    G.ws_bytes = o;

    // algorithmic HBM bytes: inputs, outputs, operands written+read, products written+read
    const double in_bytes = 4.0 * sp.w_in * (lf + lg);
    const double out_bytes = sp.mod_p ? 8.0 * G.D : 4.0 * G.w_out * G.D;
    G.hbm_bytes = in_bytes + out_bytes + 2.0 * 4.0 * G.op_limbs + 2.0 * 4.0 * npts * prod_limbs;
    G.limb_mults += G.anchor_mults;
    double norm_out = 0;
    for (auto &r : G.norms) norm_out += 4.0 * r.n_out;
    G.pack_bytes = in_bytes + 4.0 * G.op_limbs;
    const int eng0 = G.muls.empty() ? KS_ENGINE_VALU : G.muls[0].engine;
    const double col_bytes = eng0 == KS_ENGINE_MFMA ? 16.0 : 12.0;
    G.normalize_bytes = col_bytes * npts * prod_limbs + norm_out;
    G.finish_bytes = norm_out + out_bytes;
    return KS_OK;
}

// ---- profiling -----------------------------------------------------------------------------------

struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof = false;

LaunchEvents &launch_events() {
    static thread_local LaunchEvents ev;
    return ev;
}

static std::vector<ProfRec> g_prof_pending;
static std::map<std::string, std::pair<int64_t, double>> g_prof_acc;

template <class F>
static hipError_t timed(const char *name, hipStream_t s, F &&fn) {
    if (!g_prof) return fn();
    ProfRec r;
    r.name = name;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return hipErrorOutOfMemory;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipStreamIsCapturing(s, &cap);
    const bool captured = cap != hipStreamCaptureStatusNone;
    LaunchEvents &ev = launch_events();
    if (captured) hipEventRecord(r.a, s);  // a captured stream: the events bracket the region
    else ev = LaunchEvents{r.a, r.b, false};
    hipError_t e = fn();
    if (captured) {
        hipEventRecord(r.b, s);
    } else if (!ev.used) {  // nothing launched
        hipEventRecord(r.a, s);
        hipEventRecord(r.b, s);
    }
    ev = LaunchEvents{};
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back(r);
    return e;
}

hipError_t timed_launch(const char *name, hipStream_t s, const std::function<hipError_t()> &fn) {
    return timed(name, s, fn);
}

// ---- job emission (shared by single products and batches) --------------------------------------

// Append the jobs of one planned product.  f, g, h, ws are addresses (single products) or byte
// offsets from the run's bases (batches); each job's block0 continues its list.
// the look-back words of paired recombinations' second scans: after every job's own blocks
// (launched in block order), one range per paired job; returns the status words the norm list
// needs in all
int64_t assign_dual_status(JobLists &JL) {
    int64_t total = 0;
    for (const auto &j : JL.norm) total = std::max<int64_t>(total, j.block0 + j.nblocks);
    int64_t extra = 0;
    for (auto &j : JL.norm)
        if (j.dual && j.nblocks > 1) {
            j.status1 = total + extra;
            extra += j.nblocks;
        }
    return total + extra;
}

void emit_jobs(const Geom &G, uintptr_t f, uintptr_t g, uintptr_t h, uintptr_t ws, JobLists &JL) {
    const Spec &sp = G.sp;
    JL.ipt = G.ipt;  // the products of one list are planned alike (all single or all batched)
    JL.pack_ipt = G.pack_ipt;
    for (auto &m : G.muls)
        if (m.engine == KS_ENGINE_MFMA) JL.mfma_rt = m.rt;
    auto ops = [&](int64_t limb_off) { return reinterpret_cast<uint32_t *>(ws + G.ws_ops + 4 * limb_off); };
    auto cols = [&](int64_t word_off) { return reinterpret_cast<uint32_t *>(ws + G.ws_cols + 4 * word_off); };
    auto norms = [&](int64_t limb_off) { return reinterpret_cast<uint32_t *>(ws + G.ws_norms + 4 * limb_off); };
    auto anchors = [&](int64_t limb_off) { return reinterpret_cast<uint32_t *>(ws + G.ws_anchors + 4 * limb_off); };
    auto next_block = [](auto &list) -> int64_t {
        return list.empty() ? 0 : list.back().block0 + list.back().nblocks;
    };

    for (auto &p : G.packs) {
        PackJob j;
        memset(&j, 0, sizeof(j));
        j.coeffs = reinterpret_cast<const uint32_t *>(p.which ? g : f);
        j.out = ops(p.op_off);
        j.L = p.L;
        j.n_out = p.n_out;
        j.N = G.N;
        j.N_recip = div_recip((uint64_t)G.N);
        j.w_in = sp.w_in;
        j.bits = sp.bits;
        j.flags = p.flags;
        j.mod_p = sp.mod_p;
        auto &pl = p.small ? JL.pack_small : JL.pack;
        j.ctr = (int32_t)pl.size();
        j.block0 = next_block(pl);
        j.nblocks = p.blocks;
        pl.push_back(j);
    }
    auto digits = [&](int64_t byte_off) { return reinterpret_cast<uint8_t *>(ws + G.ws_digits + byte_off); };
    auto nttw = [&](int64_t word_off) { return reinterpret_cast<uint32_t *>(ws + G.ws_ntt + 4 * word_off); };
    for (auto &m : G.muls) {
        if (m.engine == KS_ENGINE_NTT) {
            const int k = m.ntt_k1 + m.ntt_k2;
            NttJob j;
            memset(&j, 0, sizeof(j));
            j.k1 = m.ntt_k1;
            j.k2 = m.ntt_k2;
            j.w = m.ntt_w;
            j.kscale[0] = ntt_scale(0, k);
            j.kscale[1] = ntt_scale(1, k);
            const int64_t per_prime = (int64_t)1 << (k - 13);  // column blocks of one prime
            for (int side = 0; side < 2; ++side) {
                NttJob f = j;
                if (side == 0) {  // the first operand's twiddles carry no factor (R in Montgomery form)
                    f.kscale[0] = (uint32_t)(((uint64_t)1 << 32) % NTT_P0);
                    f.kscale[1] = (uint32_t)(((uint64_t)1 << 32) % NTT_P1);
                }
                f.a = ops(G.packs[side ? m.fb : m.fa].op_off);
                f.na = side ? m.nb : m.na;
                f.np = side ? m.ntt_npb : m.ntt_npa;
                f.x = nttw(side ? m.ntt_xb : m.ntt_xa);
                f.nblocks = 2 * per_prime;
                f.block0 = next_block(JL.ntt_f1);
                JL.ntt_f1.push_back(f);
            }
            NttJob inv = j;
            inv.x = nttw(m.ntt_xa);
            inv.y = nttw(m.ntt_xb);
            inv.nblocks = 4 * per_prime;  // row blocks take half as many residues of each operand
            inv.block0 = next_block(JL.ntt_rows);
            JL.ntt_rows.push_back(inv);
            inv.nblocks = 2 * per_prime;
            inv.block0 = next_block(JL.ntt_i1);
            JL.ntt_i1.push_back(inv);
            NttJoinJob jj;
            memset(&jj, 0, sizeof(jj));
            jj.x = nttw(m.ntt_xa);
            jj.n = (int64_t)1 << k;
            jj.nz = m.ntt_nz;
            jj.w = m.ntt_w;
            jj.cols = nttw(m.ntt_cols);
            jj.ncols = m.ncols;
            jj.nblocks = cdiv(m.ncols, NTT_TPB);
            jj.block0 = next_block(JL.ntt_join);
            JL.ntt_join.push_back(jj);
            continue;
        }
        if (m.engine == KS_ENGINE_MFMA) {
            for (int side = 0; side < 2; ++side) {
                DigitJob d;
                memset(&d, 0, sizeof(d));
                d.limbs = ops(G.packs[side ? m.fb : m.fa].op_off);
                d.n = side ? m.nb : m.na;
                d.out = digits(side ? m.bd_off : m.ad_off);
                d.len = side ? m.b_len : m.a_len;
                d.nd = side ? m.nbd : m.nad;
                d.base = side ? m.b_top : m.a_front;
                d.reversed = side;
                d.zero = reinterpret_cast<uint8_t *>(cols(m.cols_off));
                d.zero_len = (side || m.splits * m.rgroups == 1) ? 0 : 16 * m.ncols;  // cleared for atomics only
                d.block0 = next_block(JL.digit);
                d.nblocks = cdiv(d.len + d.zero_len, 1024);
                JL.digit.push_back(d);
            }
            MfmaJob j;
            memset(&j, 0, sizeof(j));
            j.ad = digits(m.ad_off);
            j.bd = digits(m.bd_off);
            j.a_front = m.a_front;
            j.nA32 = m.nA32;
            j.b_top = m.b_top;
            j.b_len = m.b_len;
            j.nB32 = m.nB32;
            j.splits = m.splits;
            j.part = m.part;
            j.rgroups = m.rgroups;
            j.cols = reinterpret_cast<unsigned long long *>(cols(m.cols_off));
            j.block0 = next_block(JL.mfma);
            j.nblocks = m.blocks;
            JL.mfma.push_back(j);
            continue;
        }
        MulJob j;
        memset(&j, 0, sizeof(j));
        j.a = ops(G.packs[m.fa].op_off);
        j.b = ops(G.packs[m.fb].op_off);
        j.na = m.na;
        j.nb = m.nb;
        j.cols = cols(m.cols_off);
        auto &ml = m.wave ? JL.mul_wave : JL.mul;
        j.block0 = next_block(ml);
        j.nblocks = m.blocks;
        ml.push_back(j);
    }
    // the even and odd chains of the four-point reconstruction have their anchors at
    // neighbouring coefficients: for long inputs one job computes both (one stream of f and g
    // instead of two; 64-product modular batch: pack with anchors 679 -> 549 us), while short
    // ones keep a block per anchor (the 10,000-product batch lost 10 us paired), and so does a
    // single product, bound by latency
    const bool pair = sp.batch && std::min(sp.lf, sp.lg) >= 4096 && G.chains.size() == 2 && G.chains[0].step == 2 &&
                      G.chains[1].step == 2 &&
                      G.chains[0].par == 0 && G.chains[1].par == 1 && G.chains[0].K == G.chains[1].K &&
                      G.chains[1].nseg <= G.chains[0].nseg;
    for (size_t ci = 0; ci < G.chains.size(); ++ci) {
        const ChainGeom &c = G.chains[ci];
        if (c.anchor_blocks == 0 || (pair && ci == 1)) continue;
        auto &list = JL.anchor[sp.w_in];
        AnchorJob j;
        memset(&j, 0, sizeof(j));
        j.f = reinterpret_cast<const uint32_t *>(f);
        j.g = reinterpret_cast<const uint32_t *>(g);
        j.lf = sp.lf;
        j.lg = sp.lg;
        j.w_in = sp.w_in;
        j.sgn = sp.sgn;
        j.par = c.par;
        j.aw = G.aw;
        j.K = c.K;
        j.nseg = c.nseg;
        j.anchors = anchors(c.anchor_off);
        j.off_bit = G.off;
        j.kstep = c.step;
        j.anchors2 = pair ? anchors(G.chains[1].anchor_off) : j.anchors;
        j.nseg2 = pair ? G.chains[1].nseg : 0;
        j.block0 = next_block(list);
        j.nblocks = c.anchor_blocks;
        list.push_back(j);
    }
    for (auto &r : G.norms) {
        if (r.merged) continue;  // its partner's job computes it
        NormJob j;
        memset(&j, 0, sizeof(j));
        j.nterms = r.nterms;
        for (int t = 0; t < r.nterms; ++t) {
            const MulGeom &m = G.muls[r.prod[t]];
            NormTerm &T = j.term[t];
            T.cols = m.engine == KS_ENGINE_NTT ? nttw(m.ntt_cols) : cols(m.cols_off);
            T.ncols = m.ncols;
            T.a = ops(G.packs[m.fa].op_off);
            T.b = ops(G.packs[m.fb].op_off);
            T.na = m.na;
            T.nb = m.nb;
            T.sign = r.sign[t];
            T.fmt = m.engine == KS_ENGINE_MFMA ? NORM_FMT_XY : NORM_FMT_PIECES;
        }
        j.shift = r.shift;
        j.off_bit0 = r.off_bit0;
        j.off_period = r.off_period;
        j.off_recip = div_recip((uint64_t)r.off_period);
        j.off_count = r.off_count;
        j.out = norms(r.out_off);
        j.n_out = r.n_out;
        j.n_in = r.n_in;
        j.out2 = j.out;
        if (r.pair >= 0) {
            const NormGeom &r2 = G.norms[(size_t)r.pair];
            j.dual = 1;
            j.shift2 = r2.shift;
            j.sign2[0] = r2.sign[0];
            j.sign2[1] = r2.sign[1];
            j.off_bit0_2 = r2.off_bit0;
            j.off_count2 = r2.off_count;
            j.out2 = norms(r2.out_off);
            j.n_out2 = r2.n_out;
            j.n_in = std::max(r.n_in, r2.n_in);
        }
        auto &nl = r.small ? JL.norm_small : JL.norm;
        j.ctr = (int64_t)nl.size();
        j.block0 = next_block(nl);
        j.nblocks = r.blocks;
        nl.push_back(j);
    }
    for (auto &x : G.extracts) {
        ExtractJob j;
        memset(&j, 0, sizeof(j));
        j.src = norms(G.norms[x.src].out_off);
        j.n_src = G.norms[x.src].n_out;
        j.count = x.count;
        j.slot = x.slot;
        j.out = reinterpret_cast<uint32_t *>(h);
        j.out_first = x.first;
        j.out_step = x.step;
        j.w_out = G.w_out;
        j.off_bit = G.off;
        j.mod_p = sp.mod_p;
        j.block0 = next_block(JL.extract);
        j.nblocks = x.blocks;
        JL.extract.push_back(j);
    }
    for (auto &c : G.chains) {
        auto &list = JL.chain[G.nw];
        ChainJob j;
        memset(&j, 0, sizeof(j));
        j.A = norms(G.norms[c.A].out_off);
        j.nA = G.norms[c.A].n_out;
        j.B = norms(G.norms[c.B].out_off);
        j.nB = G.norms[c.B].n_out;
        j.m = c.m;
        j.K = c.K;
        j.nseg = c.nseg;
        j.anchors = anchors(c.anchor_off);
        j.aw = G.aw;
        j.Nd = (int)G.chain_nd;
        j.hbuf = reinterpret_cast<uint32_t *>(ws + G.ws_hbuf + 4 * c.hbuf_off);
        j.out = reinterpret_cast<uint32_t *>(h);
        j.out_first = c.par;
        j.out_step = c.step;
        j.w_out = G.w_out;
        j.off_bit = G.off;
        j.mod_p = sp.mod_p;
        j.block0 = next_block(list);
        j.nblocks = c.chain_blocks;
        list.push_back(j);
        // the finishing pass over the same chain: one thread per coefficient
        auto &fl = JL.finish[G.nw];
        j.block0 = next_block(fl);
        j.nblocks = c.finish_blocks;
        fl.push_back(j);
    }
}

template <class J>
static int64_t list_blocks(const std::vector<J> &v) {
    return v.empty() ? 0 : v.back().block0 + v.back().nblocks;
}

// Launch every stage of a set of job lists.  Lists of at most MAX_INLINE_JOBS jobs travel in
// the kernel arguments; longer ones need device tables (`tables`, built by a batch plan).
template <class J>
static Launch<J> make_launch(const std::vector<J> &jobs, const DevList *tab, const LaunchEnv &env, uint32_t epoch,
                             uint64_t *ctrs = nullptr) {
    Launch<J> L;
    memset(&L, 0, sizeof(L));
    L.njobs = (int64_t)jobs.size();
    L.total_blocks = list_blocks(jobs);
    if (tab) {
        L.table = reinterpret_cast<const J *>(tab->table);
        L.block_job = tab->block_job;
    } else {
        for (size_t i = 0; i < jobs.size(); ++i) L.jobs[i] = jobs[i];
    }
    L.status = env.status;
    L.ctrs = ctrs;
    L.devstat = env.devstat;
    L.epoch = epoch;
    L.base_in = env.base_in;
    L.base_out = env.base_out;
    L.base_ws = env.base_ws;
    return L;
}

int launch_lists(const JobLists &JL, const DevTables *T, const LaunchEnv &env, uint32_t epoch_pack,
                 uint32_t epoch_norm, hipStream_t s) {
    hipError_t err;
    // the first anchor list rides in the pack launch (anchors read only the inputs)
    auto first_anchor = JL.anchor.begin();
    {
        auto L = make_launch(JL.pack, T ? &T->pack : nullptr, env, epoch_pack, env.ctr_pack);
        int pack_w = 0;  // the widest input coefficient selects the pack's register layout
        for (const auto &j : JL.pack) pack_w = std::max(pack_w, (int)j.w_in);
        if (first_anchor != JL.anchor.end()) {
            auto La = make_launch(first_anchor->second, T ? &T->anchor.at(first_anchor->first) : nullptr, env, 0);
            err = timed("pack", s,
                        [&] { return launch_pack_anchor(L, La, first_anchor->first, JL.pack_ipt, pack_w, s); });
        } else {
            err = timed("pack", s, [&] { return launch_pack(L, JL.pack_ipt, pack_w, s); });
        }
        if (err != hipSuccess) return KS_EHIP;
    }
    if (!JL.pack_small.empty()) {
        auto L = make_launch(JL.pack_small, T ? &T->pack_small : nullptr, env, epoch_pack);
        int pack_w = 0;
        for (const auto &j : JL.pack_small) pack_w = std::max(pack_w, (int)j.w_in);
        err = timed("pack", s, [&] { return launch_pack_small(L, JL.pack_ipt, pack_w, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    if (!JL.mul.empty()) {
        auto L = make_launch(JL.mul, T ? &T->mul : nullptr, env, 0);
        err = timed("mul_valu", s, [&] { return launch_mul_valu(L, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    if (!JL.mul_wave.empty()) {
        auto L = make_launch(JL.mul_wave, T ? &T->mul_wave : nullptr, env, 0);
        err = timed("mul_valu", s, [&] { return launch_mul_valu_wave(L, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    if (!JL.mfma.empty()) {
        auto Ld = make_launch(JL.digit, T ? &T->digit : nullptr, env, 0);
        err = timed("digitize", s, [&] { return launch_digitize(Ld, s); });
        if (err != hipSuccess) return KS_EHIP;
        auto L = make_launch(JL.mfma, T ? &T->mfma : nullptr, env, 0);
        err = timed("mul_mfma", s, [&] { return launch_mul_mfma(L, JL.mfma_rt, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    if (!JL.ntt_f1.empty()) {
        const std::vector<NttJob> *lists[3] = {&JL.ntt_f1, &JL.ntt_rows, &JL.ntt_i1};
        const DevList *tabs[3] = {T ? &T->ntt_f1 : nullptr, T ? &T->ntt_rows : nullptr, T ? &T->ntt_i1 : nullptr};
        static const char *names[3] = {"ntt_fwd_cols", "ntt_rows", "ntt_inv_cols"};
        int max_k1 = 0, max_k2 = 0;
        for (const auto &j : JL.ntt_rows) {
            max_k1 = std::max(max_k1, (int)j.k1);
            max_k2 = std::max(max_k2, (int)j.k2);
        }
        for (int st = 0; st < 3; ++st) {
            auto L = make_launch(*lists[st], tabs[st], env, 0);
            err = timed(names[st], s, [&] { return launch_ntt_stage(st, L, max_k1, max_k2, s); });
            if (err != hipSuccess) return KS_EHIP;
        }
        auto Lj = make_launch(JL.ntt_join, T ? &T->ntt_join : nullptr, env, 0);
        err = timed("ntt_join", s, [&] { return launch_ntt_join(Lj, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    for (auto it = JL.anchor.begin(); it != JL.anchor.end(); ++it) {
        if (it == first_anchor) continue;
        const auto &kv = *it;
        auto L = make_launch(kv.second, T ? &T->anchor.at(kv.first) : nullptr, env, 0);
        err = timed("anchor", s, [&] { return launch_anchor(L, kv.first, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    {
        auto L = make_launch(JL.norm, T ? &T->norm : nullptr, env, epoch_norm, env.ctr_norm);
        bool dual = false;
        for (const auto &j : JL.norm) dual = dual || j.dual;
        err = timed("normalize", s, [&] { return launch_normalize(L, JL.ipt, dual, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    if (!JL.norm_small.empty()) {
        auto L = make_launch(JL.norm_small, T ? &T->norm_small : nullptr, env, epoch_norm);
        err = timed("normalize", s, [&] { return launch_normalize_small(L, JL.ipt, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    if (!JL.extract.empty()) {
        auto L = make_launch(JL.extract, T ? &T->extract : nullptr, env, 0);
        err = timed("extract", s, [&] { return launch_extract(L, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    for (auto &kv : JL.chain) {
        auto L = make_launch(kv.second, T ? &T->chain.at(kv.first) : nullptr, env, 0);
        err = timed("recon", s, [&] { return launch_chain(L, kv.first, T != nullptr, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    for (auto &kv : JL.finish) {
        auto L = make_launch(kv.second, T ? &T->finish.at(kv.first) : nullptr, env, 0);
        err = timed("finish", s, [&] { return launch_finish(L, kv.first, s); });
        if (err != hipSuccess) return KS_EHIP;
    }
    return KS_OK;
}

int run_product(const Geom &G, const uint32_t *f, const uint32_t *g, void *h, char *ws, Ctl &ctl, hipStream_t s) {
    for (auto &m : G.muls)
        if (m.engine == KS_ENGINE_NTT) {
            const int rc = ntt_prepare();
            if (rc != KS_OK) return rc;
            break;
        }
    JobLists JL;
    emit_jobs(G, reinterpret_cast<uintptr_t>(f), reinterpret_cast<uintptr_t>(g), reinterpret_cast<uintptr_t>(h),
              reinterpret_cast<uintptr_t>(ws), JL);
    assign_dual_status(JL);
    LaunchEnv env;
    env.status = ctl.status;
    env.ctr_pack = ctl.ctrs;
    env.ctr_norm = ctl.ctrs + CTL_CTRS;
    env.devstat = ctl.devstat;
    const uint32_t ep = ++ctl.epoch;
    const uint32_t en = ++ctl.epoch;
    return launch_lists(JL, nullptr, env, ep, en, s);
}

// ---- per-stream pools --------------------------------------------------------------------------

struct Pool {
    Ctl ctl;
    char *ws = nullptr;
    size_t bytes = 0;
    char *stage = nullptr;  // bivariate products: evaluations, univariate products, chunk sums
    size_t stage_bytes = 0;
    // bivariate products: the batch plan of their univariate products, kept while the shape
    // (length, count, modulus, inner variant) repeats
    ks_batch_plan *p2plan = nullptr;
    int64_t p2_le = 0, p2_k = 0;
    uint64_t p2_p = 0, p2_gen = 0;  // p2_gen: the tunables' generation the plan was made under
    int32_t p2_inner = -1;
};
static std::mutex g_pool_mu;
static std::map<hipStream_t, Pool *> g_pools;

static int get_pool(hipStream_t s, size_t need, int64_t status_words, Pool **out) {
    Pool *p;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto it = g_pools.find(s);
        if (it == g_pools.end()) {
            p = new Pool();
            void *c = nullptr;
            if (hipMalloc(&c, 256) != hipSuccess) { delete p; return KS_ENOMEM; }
            // cleared on the caller's stream, so the clear is ordered before this stream's kernels
            // (a non-blocking stream does not wait for work on the null stream)
            if (hipMemsetAsync(c, 0, 256, s) != hipSuccess) return KS_EHIP;
            p->ctl.ctrs = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(c) + 128);
            p->ctl.devstat = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(c) + 64);
            p->ctl.epoch = 0;
            g_pools[s] = p;
        } else {
            p = it->second;
        }
    }
    if (p->bytes < need) {
        if (p->ws) {
            if (hipStreamSynchronize(s) != hipSuccess) return KS_EHIP;
            hipFree(p->ws);
            p->ws = nullptr;
            p->bytes = 0;
        }
        size_t want = std::max<size_t>(need, (size_t)1 << 20);
        void *w = nullptr;
        if (hipMalloc(&w, want) != hipSuccess) return KS_ENOMEM;
        if (hipMemsetAsync(w, 0, want, s) != hipSuccess) return KS_EHIP;
        p->ws = reinterpret_cast<char *>(w);
        p->bytes = want;
    }
    if (p->ctl.status_words < status_words) {
        if (p->ctl.status) {
            if (hipStreamSynchronize(s) != hipSuccess) return KS_EHIP;
            hipFree(p->ctl.status);
            p->ctl.status = nullptr;
            p->ctl.status_words = 0;
        }
        const int64_t want = std::max<int64_t>(status_words, 4096);
        void *w = nullptr;
        if (hipMalloc(&w, (size_t)want * 8) != hipSuccess) return KS_ENOMEM;
        if (hipMemsetAsync(w, 0, (size_t)want * 8, s) != hipSuccess) return KS_EHIP;  // epoch 0: never fresh
        p->ctl.status = reinterpret_cast<uint64_t *>(w);
        p->ctl.status_words = want;
    }
    *out = p;
    return KS_OK;
}

int read_status(uint32_t *devstat, hipStream_t s) {
    if (hipStreamSynchronize(s) != hipSuccess) return KS_EHIP;
    uint32_t v = 0;
    if (hipMemcpy(&v, devstat, 4, hipMemcpyDeviceToHost) != hipSuccess) return KS_EHIP;
    if (v) {
        uint32_t z = 0;
        if (hipMemcpy(devstat, &z, 4, hipMemcpyHostToDevice) != hipSuccess) return KS_EHIP;
    }
    if (v & KS_DEVSTAT_RANGE) return KS_ERANGE;
    if (v & (KS_DEVSTAT_CHECK | KS_DEVSTAT_LOOKBACK)) return KS_EINTERNAL;
    return KS_OK;
}

int device_ok() {
    static int state = 0;  // 0 unknown, 1 ok, -1 not usable
    if (state == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            state = -1;
        } else {
            state = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
        }
    }
    return state;
}

int validate_spec(int64_t lf, int64_t lg, int bits, int32_t variant, bool allow_signed) {
    if (lf < 1 || lg < 1 || lf > KS_MAX_LEN || lg > KS_MAX_LEN) return KS_EINVAL;
    if (bits < 1 || bits > KS_MAX_BITS) return KS_EINVAL;
    int v = variant & KS_VARIANT_MASK;
    if (v != KS_VARIANT_AUTO && v != KS_VARIANT_KS1 && v != KS_VARIANT_NEG2 && v != KS_VARIANT_RECIP2 &&
        v != KS_VARIANT_KS4)
        return KS_EINVAL;
    if ((variant & KS_SIGNED) && !allow_signed) return KS_EINVAL;
    int known = KS_VARIANT_MASK | KS_SIGNED | KS_ENGINE_VALU | KS_ENGINE_MFMA | KS_ENGINE_NTT;
    if (variant & ~known) return KS_EINVAL;
    const int eng = variant & (KS_ENGINE_VALU | KS_ENGINE_MFMA | KS_ENGINE_NTT);
    if (eng & (eng - 1)) return KS_EINVAL;  // at most one engine
    return KS_OK;
}

int bitlen_u64(uint64_t x) {
    int n = 0;
    while (x) { ++n; x >>= 1; }
    return n;
}

}  // namespace ks

using namespace ks;

// ---- C ABI ---------------------------------------------------------------------------------------

extern "C" {

int32_t ks_version(void) { return 105; }

const char *ks_strerror(int code) {
    switch (code) {
        case KS_OK: return "ok";
        case KS_EINVAL: return "invalid argument";
        case KS_ENOMEM: return "out of memory";
        case KS_EHIP: return "HIP runtime error";
        case KS_ERANGE: return "coefficient outside its declared range";
        case KS_EUNSUPPORTED: return "not supported by this build or device";
        case KS_EINTERNAL: return "internal self-check failed";
        case KS_ESCRATCH: return "the product needs more scratch than ks_mul_noalloc's fixed array holds";
    }
    return "unknown status code";
}

int64_t ks_out_limbs(int64_t len_f, int64_t len_g, int32_t coeff_bits) {
    if (len_f < 1 || len_g < 1 || coeff_bits < 1 || coeff_bits > KS_MAX_BITS) return KS_EINVAL;
    int e = ceil_log2(std::min(len_f, len_g));
    return cdiv(2 * (int64_t)coeff_bits + e + 1, 32);
}

int ks_plan(int64_t len_f, int64_t len_g, int32_t coeff_bits, int32_t variant, ks_plan_info *out) {
    if (!out) return KS_EINVAL;
    int rc = validate_spec(len_f, len_g, coeff_bits, variant, true);
    if (rc != KS_OK) return rc;
    Spec sp{len_f, len_g, coeff_bits, (int)cdiv(coeff_bits, 32), (variant & KS_SIGNED) != 0, 0,
            variant & KS_VARIANT_MASK, variant & KS_ENGINE_ANY};
    Geom G;
    rc = plan_product(sp, G);
    if (rc != KS_OK) return rc;
    out->variant = G.variant;
    out->engine = G.muls.empty() ? KS_ENGINE_VALU : G.muls[0].engine;
    out->e = G.e;
    out->slot_bits = (int32_t)G.N;
    out->n_products = (int32_t)G.muls.size();
    out->out_limbs = G.w_out;
    out->operand_limbs_f = G.nf;
    out->operand_limbs_g = G.ng;
    out->limb_mults = G.limb_mults;
    out->schoolbook_limb_mults = G.school_mults;
    out->hbm_bytes = G.hbm_bytes;
    out->pack_bytes = G.pack_bytes;
    out->normalize_bytes = G.normalize_bytes;
    out->finish_bytes = G.finish_bytes;
    out->anchor_limb_mults = G.anchor_mults;
    out->mfma_ops = G.mfma_ops;
    out->valu_limb_mults = G.valu_mults;
    out->scratch_bytes = std::max<int64_t>(G.ws_status, (int64_t)1 << 20);  // the pool's size for it
    out->ntt_butterflies = G.ntt_butterflies;
    for (auto &m : G.muls)
        if (m.engine == KS_ENGINE_NTT) {
            out->ntt_k1 = m.ntt_k1;
            out->ntt_k2 = m.ntt_k2;
            break;
        }
    return KS_OK;
}

static int mul_common(const uint32_t *f, const uint32_t *g, const Spec &sp, void *stream, void *h) {
    if (device_ok() != 1) return KS_EUNSUPPORTED;
    Geom G;
    int rc = plan_product(sp, G);
    if (rc != KS_OK) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Pool *p = nullptr;
    // the scratch regions end where the status words would start; those live in the pool's
    // own status buffer
    rc = get_pool(s, (size_t)G.ws_status,
                  std::max<int64_t>(std::max(G.pack_blocks, G.norm_blocks + G.norm_status_extra), 1), &p);
    if (rc != KS_OK) return rc;
    return run_product(G, f, g, h, p->ws, p->ctl, s);
}

int ks_mul(const uint32_t *f, const uint32_t *g, int64_t len_f, int64_t len_g, int32_t coeff_bits, int32_t variant,
           void *stream, uint32_t *h) {
    if (!f || !g || !h) return KS_EINVAL;
    int rc = validate_spec(len_f, len_g, coeff_bits, variant, true);
    if (rc != KS_OK) return rc;
    Spec sp{len_f, len_g, coeff_bits, (int)cdiv(coeff_bits, 32), (variant & KS_SIGNED) != 0, 0,
            variant & KS_VARIANT_MASK, variant & KS_ENGINE_ANY};
    return mul_common(f, g, sp, stream, h);
}

int ks_mul_mod(const uint64_t *f, const uint64_t *g, int64_t len_f, int64_t len_g, uint64_t p, int32_t variant,
               void *stream, uint64_t *h) {
    if (!f || !g || !h) return KS_EINVAL;
    if (p < 2 || (p >> 62)) return KS_EINVAL;  // any modulus of at most 62 bits (Section 4)
    int bits = bitlen_u64(p - 1);
    int rc = validate_spec(len_f, len_g, bits, variant, false);
    if (rc != KS_OK) return rc;
    Spec sp{len_f, len_g, bits, 2, false, p, variant & KS_VARIANT_MASK, variant & KS_ENGINE_ANY};
    return mul_common(reinterpret_cast<const uint32_t *>(f), reinterpret_cast<const uint32_t *>(g), sp, stream, h);
}

// ---- bivariate products over Z/pZ (Section 2) --------------------------------------------------

int ks_mul_poly2(const uint64_t *f, const uint64_t *g, int64_t len_x, int64_t len_y, uint64_t p, int32_t variant,
                 int32_t inner, void *stream, uint64_t *h) {
    if (!f || !g || !h) return KS_EINVAL;
    if (len_x < 1 || len_y < 1 || p < 3 || !(p & 1) || (p >> 62)) return KS_EINVAL;
    if (variant & ~KS_VARIANT_MASK) return KS_EINVAL;
    if (inner & KS_SIGNED) return KS_EINVAL;
    int v = variant & KS_VARIANT_MASK;
    // a sweep over L_x = 1..256, L_y = 4..8192 (60-bit p): the standard substitution's single
    // pipeline wins below about 16K-32K residues per input (launch-bound), the four points from
    // 32K up (1.4x at 4 x 8192, 2.1x at 16 x 4096, 3.4x at 256 x 8192); at L_x = 1 the four
    // points multiply four full-length products and never win
    if (v == KS_VARIANT_AUTO) v = (len_x >= 2 && len_x * len_y >= 24576) ? KS_VARIANT_KS4 : KS_VARIANT_KS1;
    int k;
    int64_t n;
    switch (v) {
        case KS_VARIANT_KS1: k = 1; n = 2 * len_x - 1; break;       // Section 2.1
        case KS_VARIANT_RECIP2: k = 2; n = len_x; break;            // Section 2.2
        case KS_VARIANT_NEG2: k = 2; n = len_x; break;              // Section 2.3
        case KS_VARIANT_KS4: k = 4; n = (len_x + 1) / 2; break;     // Section 2.4
        case KS_P2_COMPLEX: k = 5; n = (len_x + 1) / 2; break;      // Section 2.5, y = x^M, -x^M, i x^M
        case KS_P2_CUBE:                                            // Section 2.5, y = +-x^M, +-w x^M
            if (p % 3 == 0) return KS_EINVAL;                       // divides by 6
            k = 8;
            n = (len_x + 2) / 3;
            break;
        default: return KS_EINVAL;
    }
    const bool ext = v == KS_P2_COMPLEX || v == KS_P2_CUBE;
    const int64_t le = n * (len_y - 1) + len_x, lh = 2 * le - 1;
    if (le > (int64_t)1 << 30) return KS_EINVAL;
    const int bits = bitlen_u64(p - 1);
    int rc = validate_spec(le, le, bits, inner, false);
    if (rc != KS_OK) return rc;
    if (device_ok() != 1) return KS_EUNSUPPORTED;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Pool *pl = nullptr;
    rc = get_pool(s, 0, 1, &pl);
    if (rc != KS_OK) return rc;
    // two or four univariate products run as one batch (one set of launches: 0.82 -> 0.56 ms on
    // the 16 x 4096 four-point workload), its plan cached per stream; arena offsets (uint32
    // limbs) from the stage, evaluations first, then the products.  A single product keeps the
    // single-product pipeline (reconstruction segments cut for latency: 1.16 against 1.22 ms)
    // unless it is long enough for the batch plan's Karatsuba split.
    ks_desc d[8];
    memset(d, 0, sizeof(d));
    for (int q = 0; q < k; ++q) {
        d[q].f_off = (uint64_t)(2 * q * le);
        d[q].g_off = (uint64_t)(2 * (k + q) * le);
        d[q].h_off = (uint64_t)(2 * (2 * k * le + q * lh));
        d[q].len_f = (int32_t)le;
        d[q].len_g = (int32_t)le;
        d[q].coeff_bits = bits;
        d[q].flags = KS_MOD;
        d[q].mod_p = p;
    }
    const bool batched = k > 1 || karatsuba_splits(d, k, inner);
    const uint64_t gen = tune_generation();
    if (batched && (!pl->p2plan || pl->p2_le != le || pl->p2_k != k || pl->p2_p != p || pl->p2_inner != inner ||
                    pl->p2_gen != gen)) {
        if (pl->p2plan) {
            if (hipStreamSynchronize(s) != hipSuccess) return KS_EHIP;  // its tables may be in use
            ks_batch_plan_destroy(pl->p2plan);
            pl->p2plan = nullptr;
        }
        rc = ks_batch_plan_create(d, k, inner, &pl->p2plan);
        if (rc != KS_OK) return rc;
        pl->p2_le = le;
        pl->p2_k = k;
        pl->p2_p = p;
        pl->p2_inner = inner;
        pl->p2_gen = gen;
    }
    // stage: 2k evaluations, k products, chunk sums of up to two gluings, the batch workspace
    const int64_t m = v == KS_VARIANT_KS4 ? 2 * n : n, count = v == KS_VARIANT_KS4 ? len_y : 2 * len_y - 1;
    const int64_t nchunks = ext ? 0 : cdiv((count + 1) / 2, P2_CHUNK);
    const int64_t words = 2 * k * le + k * lh + 2 * nchunks * 4 * m;
    const size_t ws_off = ((size_t)words * 8 + 255) / 256 * 256;
    const size_t need = ws_off + (batched ? ks_batch_plan_workspace_bytes(pl->p2plan) : 0);
    if (pl->stage_bytes < need) {
        if (pl->stage) {
            if (hipStreamSynchronize(s) != hipSuccess) return KS_EHIP;
            hipFree(pl->stage);
            pl->stage = nullptr;
            pl->stage_bytes = 0;
        }
        void *w = nullptr;
        if (hipMalloc(&w, need) != hipSuccess) return KS_ENOMEM;
        pl->stage = reinterpret_cast<char *>(w);
        pl->stage_bytes = need;
    }
    uint64_t *ev = reinterpret_cast<uint64_t *>(pl->stage), *prod = ev + 2 * k * le, *sums = prod + k * lh;
    if (ext) {
        // the evaluations: the points' components as small integer weights of the rows
        // (period 4 for i^row, 3 for w^row, 6 for (-w)^row), and the sums of the two components
        // that the ring products' middle terms multiply
        P2ExtEval E;
        memset(&E, 0, sizeof(E));
        E.f = f;
        E.g = g;
        E.out = ev;
        E.lx = len_x;
        E.ly = len_y;
        E.m = n;
        E.le = le;
        E.p = p;
        E.np = k;
        E.devstat = pl->ctl.devstat;
        static const int8_t cplx[5][4] = {{1, 1, 1, 1},     // y = x^M
                                          {1, -1, 1, -1},   // y = -x^M
                                          {1, 0, -1, 0},    // real part of i^row
                                          {0, 1, 0, -1},    // imaginary part
                                          {1, 1, -1, -1}};  // their sum
        static const int8_t cube[8][6] = {{1, 1, 1, 1, 1, 1},       // y = x^M
                                          {1, -1, 1, -1, 1, -1},    // y = -x^M
                                          {1, 0, -1, 1, 0, -1},     // w^row = a + b w: a
                                          {0, 1, -1, 0, 1, -1},     //                  b
                                          {1, 1, -2, 1, 1, -2},     //                  a + b
                                          {1, 0, -1, -1, 0, 1},     // (-w)^row: a
                                          {0, -1, -1, 0, 1, 1},     //           b
                                          {1, -1, -2, -1, 1, 2}};   //           a + b
        E.period = v == KS_P2_COMPLEX ? 4 : 6;
        for (int q = 0; q < k; ++q)
            for (int i = 0; i < E.period; ++i) E.coef[q][i] = v == KS_P2_COMPLEX ? cplx[q][i] : cube[q][i];
        if (timed("p2_eval", s, [&] { return launch_p2_ext_eval(E, s); }) != hipSuccess) return KS_EHIP;
        rc = batch_run_into(pl->p2plan, reinterpret_cast<const uint32_t *>(pl->stage),
                            reinterpret_cast<uint32_t *>(pl->stage), pl->stage + ws_off, pl->ctl.devstat, s);
        if (rc != KS_OK) return rc;
        P2ExtReadoff R;
        memset(&R, 0, sizeof(R));
        R.prod = prod;
        R.out = h;
        R.lh = lh;
        R.rows = 2 * len_y - 1;
        R.width = 2 * len_x - 1;
        R.m = n;
        R.p = p;
        R.cube = v == KS_P2_CUBE;
        const uint64_t d4 = v == KS_P2_COMPLEX ? 4 : 6;  // its inverse mod p by Euclid
        {
            __int128 t0 = 0, t1 = 1, r0 = (__int128)p, r1 = (__int128)(d4 % p);
            while (r1 != 0) {
                const __int128 qq = r0 / r1, t2 = t0 - qq * t1, r2 = r0 - qq * r1;
                t0 = t1;
                t1 = t2;
                r0 = r1;
                r1 = r2;
            }
            R.inv = (uint64_t)(t0 < 0 ? t0 + (__int128)p : t0);
        }
        const hipError_t e2 = timed("p2_recon", s, [&] { return launch_p2_ext_readoff(R, s); });
        return e2 == hipSuccess ? KS_OK : KS_EHIP;
    }
    P2Eval E;
    memset(&E, 0, sizeof(E));
    E.f = f;
    E.g = g;
    E.out = ev;
    E.lx = len_x;
    E.ly = len_y;
    E.n = n;
    E.le = le;
    E.p = p;
    E.k = k;
    E.devstat = pl->ctl.devstat;
    // evaluation points in the order of the products: x^N, then -x^N or x^-N (two points),
    // or x^N, -x^N, x^-N, -x^-N (four)
    for (int q = 0; q < k; ++q) {
        E.neg[q] = (v == KS_VARIANT_NEG2 && q == 1) || (v == KS_VARIANT_KS4 && (q & 1));
        E.rev[q] = (v == KS_VARIANT_RECIP2 && q == 1) || (v == KS_VARIANT_KS4 && q >= 2);
    }
    if (timed("p2_eval", s, [&] { return launch_p2_eval(E, s); }) != hipSuccess) return KS_EHIP;
    if (batched) {
        rc = batch_run_into(pl->p2plan, reinterpret_cast<const uint32_t *>(pl->stage),
                            reinterpret_cast<uint32_t *>(pl->stage), pl->stage + ws_off, pl->ctl.devstat, s);
    } else {
        Spec sp{le, le, bits, 2, false, p, inner & KS_VARIANT_MASK, inner & KS_ENGINE_ANY};
        rc = mul_common(reinterpret_cast<const uint32_t *>(ev), reinterpret_cast<const uint32_t *>(ev + le), sp,
                        stream, prod);
    }
    if (rc != KS_OK) return rc;
    auto side = [&](int a, int b, int comb, int64_t off) {
        P2Side S;
        memset(&S, 0, sizeof(S));
        S.x = prod + a * lh;
        S.y = b >= 0 ? prod + b * lh : nullptr;
        S.len = lh;
        S.off = off;
        S.comb = comb;
        return S;
    };
    const int64_t width = 2 * len_x - 1, rows = 2 * len_y - 1;
    hipError_t err = hipSuccess;
    if (v == KS_VARIANT_KS1 || v == KS_VARIANT_NEG2) {
        P2Readoff R;
        memset(&R, 0, sizeof(R));
        R.even = v == KS_VARIANT_KS1 ? side(0, -1, 0, 0) : side(0, 1, 1, 0);
        R.odd = v == KS_VARIANT_KS1 ? side(0, -1, 0, 0) : side(0, 1, -1, 0);
        R.out = h;
        R.rows = rows;
        R.width = width;
        R.n = n;
        R.p = p;
        err = timed("p2_recon", s, [&] { return launch_p2_readoff(R, s); });
    } else {
        P2Glue G;
        memset(&G, 0, sizeof(G));
        G.out = h;
        G.m = m;
        G.width = width;
        G.p = p;
        G.devstat = pl->ctl.devstat;
        auto part = [&](int i, P2Side A, P2Side B, int64_t cnt, int64_t row0, int64_t rstep) {
            P2GluePart &P = G.part[i];
            P.A = A;
            P.B = B;
            P.sums = sums + i * nchunks * 4 * m;
            P.count = cnt;
            P.row0 = row0;
            P.rstep = rstep;
            P.nchunks = cdiv((cnt + 1) / 2, P2_CHUNK);
            G.nparts = i + 1;
        };
        if (v == KS_VARIANT_RECIP2) {
            part(0, side(0, -1, 0, 0), side(1, -1, 0, 0), rows, 0, 1);
        } else {
            // even part (H1 + H2) / 2 and (H3 + H4) / 2, odd part the halved differences / x^N
            part(0, side(0, 1, 1, 0), side(2, 3, 1, 0), len_y, 0, 2);
            if (len_y > 1) part(1, side(0, 1, -1, n), side(2, 3, -1, n), len_y - 1, 1, 2);
        }
        err = timed("p2_recon", s, [&] { return launch_p2_glue(G, s); });
    }
    return err == hipSuccess ? KS_OK : KS_EHIP;
}

int ks_stream_status(void *stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Pool *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto it = g_pools.find(s);
        if (it != g_pools.end()) p = it->second;
    }
    int rc = p ? read_status(p->ctl.devstat, s) : (hipStreamSynchronize(s) == hipSuccess ? KS_OK : KS_EHIP);
    const int rc2 = noalloc_status(s);  // ks_mul_noalloc's status word on this device
    return rc != KS_OK ? rc : rc2;
}

int ks_profile_enable(int32_t on) {
    g_prof = on != 0;
    return KS_OK;
}

int ks_tune_set(const char *name, int64_t value) {
    if (!name || !known_tunable(name) || value < 0) return KS_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[name] = value;
    ++g_tune_gen;  // cached plans (the bivariate products') are made again
    return KS_OK;
}

int ks_tune_get(const char *name, int64_t *value) {
    if (!name || !value || !known_tunable(name)) return KS_EINVAL;
    static const int dflt[] = {2500, 0, 128, 10, 0, 128, (int)small_bl(SCAN_IPT_SINGLE), 0,
                               KARATSUBA_MIN_LIMBS, NTT_MIN_LIMBS, SCAN_BIG_LIMBS};  // as for a single product
    int d = 0;
    for (size_t q = 0; q < sizeof(k_tunables) / sizeof(k_tunables[0]); ++q)
        if (strcmp(k_tunables[q], name) == 0) d = dflt[q];
    *value = env_int(name, d);
    return KS_OK;
}

int ks_tune_reset(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    ++g_tune_gen;
    return KS_OK;
}

int ks_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof_pending) {
        hipEventSynchronize(r.b);
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    g_prof_acc.clear();
    return KS_OK;
}

int ks_profile_read(const char *name, int64_t *launches, double *total_ms) {
    if (!name || !launches || !total_ms) return KS_EINVAL;
    static const char *known[] = {"pack",  "mul_valu", "mul_mfma", "normalize", "anchor",  "recon",
                                  "extract", "digitize", "finish",  "p2_eval",   "p2_recon", "kara",
                                  "ntt_fwd_cols", "ntt_rows", "ntt_inv_cols", "ntt_join"};
    bool ok = false;
    for (const char *k : known) ok = ok || strcmp(k, name) == 0;
    if (!ok) return KS_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof_pending) {
        if (hipEventSynchronize(r.b) != hipSuccess) return KS_EHIP;
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.a, r.b);
        auto &acc = g_prof_acc[r.name];
        acc.first += 1;
        acc.second += ms;
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    auto it = g_prof_acc.find(name);
    *launches = it == g_prof_acc.end() ? 0 : it->second.first;
    *total_ms = it == g_prof_acc.end() ? 0.0 : it->second.second;
    return KS_OK;
}

}  // extern "C"

