/*
 * oracle.c -- exact CPU oracle for dense products in Z[x] and (Z/pZ)[x].
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls this file;
 * only the test-suite, the smoke check and the benchmark's CPU-baseline leg do.  It shares
 * no code, header or table with the GPU path.
 *
 * What it computes (paper, Section 3, opening paragraph): for f, g in Z[x] of lengths
 * len_f, len_g, the product h = f g with D = len_f + len_g - 1 coefficients
 *     h_k = sum_{i + j = k} f_i g_j .
 * Two independent routes:
 *   or_mul_classical -- that definition written out, coefficient by coefficient, with
 *                       fixed-width two's-complement multi-limb accumulators;
 *   or_mul_ks1       -- standard Kronecker substitution (Section 3.1): evaluate both inputs
 *                       at 2^N with N = 2b + e, multiply the two integers with a schoolbook
 *                       bignum, and read the coefficients back off the product's bits.
 *                       Signed inputs (not covered by the paper) are read off as balanced
 *                       base-2^N digits: |h_k| <= L 2^(2b-2) < 2^(N-1), so each digit is
 *                       unique in [-2^(N-1), 2^(N-1)).
 * and reduction modulo any p with 2 <= p < 2^63 (Section 4: lift to Z[x], multiply, reduce).
 *
 * Coefficient layout: coefficient i occupies w consecutive little-endian 32-bit limbs; when
 * is_signed is set the limbs hold the two's complement of the value.  Outputs use the same
 * layout with w_out limbs (two's complement).
 *
 * Every function returns 0 on success and a negative number on bad arguments.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXW 512 /* largest limb count handled for one coefficient or accumulator */

/* ---- fixed-width multi-limb helpers (wrapping, i.e. modulo 2^(32 n)) ---------------------- */

/* acc += x  (x has m limbs, missing limbs are zero) */
static void mp_add(uint32_t *acc, int n, const uint32_t *x, int m)
{
    uint64_t c = 0;
    for (int i = 0; i < n; i++) {
        uint64_t s = (uint64_t)acc[i] + (i < m ? x[i] : 0u) + c;
        acc[i] = (uint32_t)s;
        c = s >> 32;
    }
}

/* acc -= x */
static void mp_sub(uint32_t *acc, int n, const uint32_t *x, int m)
{
    uint64_t br = 0;
    for (int i = 0; i < n; i++) {
        uint64_t d = (uint64_t)acc[i] - (i < m ? x[i] : 0u) - br;
        acc[i] = (uint32_t)d;
        br = (d >> 63) & 1u;
    }
}

/* x = -x */
static void mp_neg(uint32_t *x, int n)
{
    uint64_t c = 1;
    for (int i = 0; i < n; i++) {
        uint64_t s = (uint64_t)(uint32_t)~x[i] + c;
        x[i] = (uint32_t)s;
        c = s >> 32;
    }
}

/* out (na + nb limbs) = a * b, schoolbook */
static void mp_mul(uint32_t *out, const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb)
{
    memset(out, 0, sizeof(uint32_t) * (size_t)(na + nb));
    for (int64_t i = 0; i < na; i++) {
        uint64_t c = 0;
        uint64_t ai = a[i];
        for (int64_t j = 0; j < nb; j++) {
            uint64_t t = ai * b[j] + out[i + j] + c;
            out[i + j] = (uint32_t)t;
            c = t >> 32;
        }
        out[i + nb] = (uint32_t)c;
    }
}

/* Split a w-limb coefficient into magnitude (w limbs) and sign. */
static int coeff_mag(const uint32_t *c, int w, int is_signed, uint32_t *mag)
{
    memcpy(mag, c, sizeof(uint32_t) * (size_t)w);
    if (is_signed && (c[w - 1] >> 31)) {
        mp_neg(mag, w);
        return 1;
    }
    return 0;
}

static int ceil_log2_i64(int64_t x)
{
    int e = 0;
    while (((int64_t)1 << e) < x) e++;
    return e;
}

/* ---- route 1: the plain definition ------------------------------------------------------- */

static void classical_one(const uint32_t *fm, const uint8_t *fs, const uint32_t *gm,
                          const uint8_t *gs, int64_t lf, int64_t lg, int w, int64_t k,
                          uint32_t *acc, int w_out)
{
    uint32_t prod[2 * 64];
    memset(acc, 0, sizeof(uint32_t) * (size_t)w_out);
    int64_t lo = k - (lg - 1) > 0 ? k - (lg - 1) : 0;
    int64_t hi = k < lf - 1 ? k : lf - 1;
    for (int64_t i = lo; i <= hi; i++) {
        int64_t j = k - i;
        mp_mul(prod, fm + i * w, w, gm + j * w, w);
        if (fs[i] ^ gs[j])
            mp_sub(acc, w_out, prod, 2 * w);
        else
            mp_add(acc, w_out, prod, 2 * w);
    }
}

/* split inputs into magnitudes and signs (caller frees) */
static int split_inputs(const uint32_t *c, int64_t len, int w, int is_signed, uint32_t **mag,
                        uint8_t **sg)
{
    *mag = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(len * w));
    *sg = (uint8_t *)malloc((size_t)len);
    if (!*mag || !*sg) return -2;
    for (int64_t i = 0; i < len; i++) (*sg)[i] = (uint8_t)coeff_mag(c + i * w, w, is_signed, *mag + i * w);
    return 0;
}

/* h[k] for every k in [0, D), D = lf + lg - 1 */
int or_mul_classical(const uint32_t *f, const uint32_t *g, int64_t lf, int64_t lg, int w_in,
                     int is_signed, uint32_t *h, int w_out)
{
    if (lf < 1 || lg < 1 || w_in < 1 || w_in > 64 || w_out < 1 || w_out > OR_MAXW) return -1;
    uint32_t *fm, *gm;
    uint8_t *fs, *gs;
    if (split_inputs(f, lf, w_in, is_signed, &fm, &fs) || split_inputs(g, lg, w_in, is_signed, &gm, &gs))
        return -2;
    int64_t D = lf + lg - 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < D; k++) classical_one(fm, fs, gm, gs, lf, lg, w_in, k, h + k * w_out, w_out);
    free(fm); free(fs); free(gm); free(gs);
    return 0;
}

/* h[ks[t]] for a list of indices (used for sampled checks of very large products) */
int or_coeffs_classical(const uint32_t *f, const uint32_t *g, int64_t lf, int64_t lg, int w_in,
                        int is_signed, const int64_t *ks, int64_t nk, uint32_t *out, int w_out)
{
    if (lf < 1 || lg < 1 || w_in < 1 || w_in > 64 || w_out < 1 || w_out > OR_MAXW) return -1;
    uint32_t *fm, *gm;
    uint8_t *fs, *gs;
    if (split_inputs(f, lf, w_in, is_signed, &fm, &fs) || split_inputs(g, lg, w_in, is_signed, &gm, &gs))
        return -2;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nk; t++) {
        if (ks[t] < 0 || ks[t] >= lf + lg - 1) { bad = 1; continue; }
        classical_one(fm, fs, gm, gs, lf, lg, w_in, ks[t], out + t * w_out, w_out);
    }
    free(fm); free(fs); free(gm); free(gs);
    return bad ? -1 : 0;
}

/* ---- route 2: standard Kronecker substitution over a schoolbook bignum -------------------- */

/* big (n limbs, two's complement, wrapping) += s * mag * 2^shift, mag has w limbs */
static void add_shifted(uint32_t *big, int64_t n, const uint32_t *mag, int w, int negate,
                        int64_t shift)
{
    int64_t q = shift / 32;
    int r = (int)(shift % 32);
    uint32_t tmp[65];
    for (int t = 0; t <= w; t++) {
        uint32_t lo = t < w ? mag[t] : 0u;
        uint32_t prev = t > 0 ? mag[t - 1] : 0u;
        tmp[t] = r ? (lo << r) | (prev >> (32 - r)) : lo;
    }
    /* add or subtract tmp at limb offset q, propagating to the top only while needed */
    uint64_t c = 0;
    for (int64_t i = q; i < n; i++) {
        int64_t t = i - q;
        uint32_t x = t <= w ? tmp[t] : 0u;
        if (t > w && c == 0) break;
        if (!negate) {
            uint64_t s = (uint64_t)big[i] + x + c;
            big[i] = (uint32_t)s;
            c = s >> 32;
        } else {
            uint64_t d = (uint64_t)big[i] - x - c;
            big[i] = (uint32_t)d;
            c = (d >> 63) & 1u;
        }
    }
}

/* bits [start, start + len) of x (n limbs, two's complement, sign-extended) into out (wo limbs) */
static void get_bits(const uint32_t *x, int64_t n, int64_t start, int len, uint32_t *out, int wo)
{
    uint32_t sx = (x[n - 1] >> 31) ? 0xffffffffu : 0u;
    memset(out, 0, sizeof(uint32_t) * (size_t)wo);
    for (int b = 0; b < len; b++) {
        int64_t pos = start + b;
        int64_t li = pos / 32;
        uint32_t word = li < n ? x[li] : sx;
        if ((word >> (pos % 32)) & 1u) out[b / 32] |= 1u << (b % 32);
    }
}

static int test_bit(const uint32_t *x, int bit) { return (x[bit / 32] >> (bit % 32)) & 1u; }

int or_mul_ks1(const uint32_t *f, const uint32_t *g, int64_t lf, int64_t lg, int w_in, int b,
               int is_signed, uint32_t *h, int w_out)
{
    if (lf < 1 || lg < 1 || w_in < 1 || w_in > 64 || b < 1 || b > 32 * w_in || w_out < 1 ||
        w_out > OR_MAXW)
        return -1;
    int e = ceil_log2_i64(lf < lg ? lf : lg);
    int64_t N = 2 * (int64_t)b + e; /* Section 3.1 */
    int64_t nF = (N * (lf - 1) + b + 33) / 32 + 1;
    int64_t nG = (N * (lg - 1) + b + 33) / 32 + 1;
    uint32_t *F = (uint32_t *)calloc((size_t)nF, 4), *G = (uint32_t *)calloc((size_t)nG, 4);
    uint32_t *H = (uint32_t *)calloc((size_t)(nF + nG), 4);
    uint32_t mag[64];
    if (!F || !G || !H) return -2;
    /* evaluation at 2^N: F = sum f_i 2^(iN) */
    for (int64_t i = 0; i < lf; i++) {
        int s = coeff_mag(f + i * w_in, w_in, is_signed, mag);
        add_shifted(F, nF, mag, w_in, s, N * i);
    }
    for (int64_t i = 0; i < lg; i++) {
        int s = coeff_mag(g + i * w_in, w_in, is_signed, mag);
        add_shifted(G, nG, mag, w_in, s, N * i);
    }
    /* one integer product, through magnitudes */
    int sF = (int)(F[nF - 1] >> 31), sG = (int)(G[nG - 1] >> 31);
    if (sF) mp_neg(F, (int)nF);
    if (sG) mp_neg(G, (int)nG);
    mp_mul(H, F, nF, G, nG);
    if (sF ^ sG) mp_neg(H, (int)(nF + nG));
    /* unpack: coefficient k is digit k of H in base 2^N */
    int64_t D = lf + lg - 1;
    int wv = (int)(N / 32) + 2;
    uint32_t v[OR_MAXW + 2], one[1] = {1u};
    if (wv > OR_MAXW) return -1;
    int carry = 0;
    for (int64_t k = 0; k < D; k++) {
        get_bits(H, nF + nG, k * N, (int)N, v, wv);
        if (carry) mp_add(v, wv, one, 1);
        carry = 0;
        if (is_signed && (test_bit(v, (int)N) || test_bit(v, (int)N - 1))) {
            /* balanced digit: v - 2^N, with a carry into the next digit */
            uint32_t pw[OR_MAXW + 2];
            memset(pw, 0, sizeof(uint32_t) * (size_t)wv);
            pw[N / 32] = 1u << (N % 32);
            mp_sub(v, wv, pw, wv);
            carry = 1;
        }
        uint32_t sx = (is_signed && (v[wv - 1] >> 31)) ? 0xffffffffu : 0u;
        for (int t = 0; t < w_out; t++) h[k * w_out + t] = t < wv ? v[t] : sx;
    }
    free(F); free(G); free(H);
    return 0;
}

/* ---- reduction modulo p (Section 4) ------------------------------------------------------- */

typedef unsigned __int128 u128;

/* h_k mod p for one k; inputs are residues in [0, p), 2 <= p < 2^63 */
static uint64_t coeff_mod_one(const uint64_t *f, const uint64_t *g, int64_t lf, int64_t lg,
                              uint64_t p, int64_t k)
{
    int64_t lo = k - (lg - 1) > 0 ? k - (lg - 1) : 0;
    int64_t hi = k < lf - 1 ? k : lf - 1;
    u128 acc = 0;
    int cnt = 0;
    for (int64_t i = lo; i <= hi; i++) {
        acc += (u128)f[i] * g[k - i]; /* each term < 2^126 */
        if (++cnt == 2) { acc %= p; cnt = 0; }
    }
    return (uint64_t)(acc % p);
}

int or_mul_mod(const uint64_t *f, const uint64_t *g, int64_t lf, int64_t lg, uint64_t p, uint64_t *h)
{
    if (lf < 1 || lg < 1 || p < 2 || (p >> 63)) return -1;
    for (int64_t i = 0; i < lf; i++) if (f[i] >= p) return -1;
    for (int64_t i = 0; i < lg; i++) if (g[i] >= p) return -1;
    int64_t D = lf + lg - 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < D; k++) h[k] = coeff_mod_one(f, g, lf, lg, p, k);
    return 0;
}

int or_coeffs_mod(const uint64_t *f, const uint64_t *g, int64_t lf, int64_t lg, uint64_t p,
                  const int64_t *ks, int64_t nk, uint64_t *out)
{
    if (lf < 1 || lg < 1 || p < 2 || (p >> 63)) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nk; t++) {
        if (ks[t] < 0 || ks[t] >= lf + lg - 1) { bad = 1; continue; }
        out[t] = coeff_mod_one(f, g, lf, lg, p, ks[t]);
    }
    return bad ? -1 : 0;
}

/* number of OpenMP threads the parallel loops above use (1 when built without OpenMP) */
int or_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
