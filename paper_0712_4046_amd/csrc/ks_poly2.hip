// ks_poly2.hip -- bivariate products over Z/pZ by Kronecker substitution into (Z/pZ)[x]
// (paper Section 2).  f, g in (Z/pZ)[x, y] are evaluated at y = +-x^N or (normalised)
// +-x^-N (p2_eval_kernel), the univariate products are the library's modular products, and
// h is recovered from them by reading off (standard substitution), halving (negated points)
// and the gluing of overlapping halves (reciprocal points; p2_glue_*).
//
// Residues are uint64 in [0, p), p odd and below 2^62, so a sum of two stays below 2^63.
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

__device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t p) {
    const uint64_t s = a + b;
    return s >= p ? s - p : s;
}
__device__ __forceinline__ uint64_t sub_mod_p(uint64_t a, uint64_t b, uint64_t p) { return a >= b ? a - b : a + p - b; }
// s / 2 in Z/pZ (p odd)
__device__ __forceinline__ uint64_t half_mod(uint64_t s, uint64_t p) { return (s & 1) ? (s + p) >> 1 : s >> 1; }

// ---- evaluation ---------------------------------------------------------------------------------

// Position i N + r of evaluation q of input w (f, then g): sum over the rows that reach it,
// row i - t at column r + t N (Section 2.4: rows overlap when N < L_x), each row taken in
// reversed order for the reciprocal points and negated at odd i for the negated points.
__global__ __launch_bounds__(256) void p2_eval_kernel(P2Eval E) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= 2 * E.k * E.le) return;
    const int64_t wq = t / E.le, pos = t - wq * E.le;
    const int w = (int)(wq / E.k), q = (int)(wq - (int64_t)w * E.k);
    const uint64_t *src = w ? E.g : E.f;
    const int64_t i = pos / E.n, r = pos - i * E.n;
    uint64_t acc = 0;
    bool bad = false;
    for (int64_t s = 0; i - s >= 0 && r + s * E.n < E.lx; ++s) {
        const int64_t row = i - s;
        if (row >= E.ly) continue;
        const int64_t srow = E.rev[q] ? E.ly - 1 - row : row;
        uint64_t v = src[srow * E.lx + r + s * E.n];
        bad |= v >= E.p;
        if (E.neg[q] && (row & 1)) v = v ? E.p - v : 0;
        acc = add_mod(acc, v, E.p);
    }
    if (bad) set_status(E.devstat, KS_DEVSTAT_RANGE);
    E.out[wq * E.le + pos] = acc;
}

// ---- recovery -------------------------------------------------------------------------------------

// value at position pos of a side: a product, or half the sum or difference of two, shifted
__device__ __forceinline__ uint64_t side_at(const P2Side &S, int64_t pos, uint64_t p) {
    pos += S.off;
    if (pos < 0 || pos >= S.len) return 0;
    const uint64_t a = S.x[pos];
    if (S.comb == 0) return a;
    const uint64_t b = S.y[pos];
    return half_mod(S.comb > 0 ? add_mod(a, b, p) : sub_mod_p(a, b, p), p);
}

// Standard and negated substitutions: h_k[c] = side(k N + c), the side chosen by the parity
// of k (the negated points' even part (H+ + H-)/2 and odd part (H+ - H-)/2 at x^N: Sections
// 2.1 and 2.3)
__global__ __launch_bounds__(256) void p2_readoff_kernel(P2Readoff R) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= R.rows * R.width) return;
    const int64_t k = t / R.width, c = t - k * R.width;
    R.out[t] = side_at((k & 1) ? R.odd : R.even, k * R.n + c, R.p);
}

// Gluing (Section 2.2) of u_0 .. u_(D-1), each of at most 2M - 1 coefficients, from
// A = sum_j u_j x^(j M) and B = sum_j u_(D-1-j) x^(j M).  With a_j the low M coefficients of
// u_j and b_j the next M - 1, position j M + r of A holds a_j[r] + b_(j-1)[r] and position
// (D - j) M + r of B holds b_j[r] + a_(j-1)[r], so for r < M - 1
//   a_j = A_j - B'_(j-1) + a_(j-2),   b_j = B'_j - A_(j-1) + b_(j-2)
// (A_j[r] = A(j M + r), B'_j[r] = B((D - j) M + r)): each of a, b is a prefix sum over the
// steps j of one parity.  Position j M + M - 1 of A holds a_j[M - 1] alone (u_(j-1) has no
// coefficient 2M - 1), so that column is read off.  Sequence s = (kind, parity, r); its steps
// are cut into chunks of P2_CHUNK: p2_glue_sum_kernel sums each chunk, p2_glue_scan_kernel
// turns each sequence's chunk sums into exclusive prefixes, p2_glue_out_kernel writes the
// chunk's steps from its prefix.  Coefficients at or above the output width must come out
// zero (a free check of the recovery).
__device__ __forceinline__ uint64_t glue_term(const P2GluePart &G, int64_t m, uint64_t p, int kind, int64_t j,
                                              int64_t r) {
    auto Bp = [&](int64_t jj) -> uint64_t {
        return (jj >= 0 && r < m - 1) ? side_at(G.B, (G.count - jj) * m + r, p) : 0;
    };
    if (kind == 0) return sub_mod_p(side_at(G.A, j * m + r, p), Bp(j - 1), p);
    if (r >= m - 1) return 0;
    return sub_mod_p(Bp(j), j >= 1 ? side_at(G.A, (j - 1) * m + r, p) : 0, p);
}

struct GlueUnit {
    int part, kind, par;
    int64_t s, r, chunk, t0, t1;  // steps j = par + 2 t, t in [t0, t1)
};
// unit u of a launch: chunk-major within each part, the 4M sequences of a chunk fastest
__device__ __forceinline__ bool glue_unit(const P2Glue &G, int64_t u, GlueUnit &U) {
    const int64_t nseq = 4 * G.m;
    U.part = 0;
    if (u >= G.part[0].nchunks * nseq) {
        u -= G.part[0].nchunks * nseq;
        U.part = 1;
        if (G.nparts < 2 || u >= G.part[1].nchunks * nseq) return false;
    }
    const P2GluePart &P = G.part[U.part];
    U.chunk = u / nseq;
    U.s = u - U.chunk * nseq;
    const int64_t kp = U.s / G.m;
    U.r = U.s - kp * G.m;
    U.kind = (int)(kp >> 1);
    U.par = (int)(kp & 1);
    const int64_t steps = (P.count - U.par + 1) / 2;  // j = par, par + 2, ... < count
    U.t0 = U.chunk * P2_CHUNK;
    U.t1 = U.t0 + P2_CHUNK < steps ? U.t0 + P2_CHUNK : steps;
    return true;
}

__global__ __launch_bounds__(256) void p2_glue_sum_kernel(P2Glue G) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    GlueUnit U;
    if (!glue_unit(G, u, U)) return;
    const P2GluePart &P = G.part[U.part];
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < P2_CHUNK; ++q)
        if (U.t0 + q < U.t1) acc = add_mod(acc, glue_term(P, G.m, G.p, U.kind, U.par + 2 * (U.t0 + q), U.r), G.p);
    P.sums[U.chunk * 4 * G.m + U.s] = acc;
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t x, int d) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, 64);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// one wave per (part, sequence): its chunk sums to exclusive prefixes, in place, 64 chunks
// per round (a wave-wide inclusive scan plus the carry of the rounds before)
__global__ __launch_bounds__(256) void p2_glue_scan_kernel(P2Glue G) {
    const int lane = threadIdx.x & 63;
    int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nseq = 4 * G.m;
    int part = 0;
    if (u >= nseq) {
        u -= nseq;
        part = 1;
        if (G.nparts < 2 || u >= nseq) return;  // wave-uniform
    }
    const P2GluePart &P = G.part[part];
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < P.nchunks; c0 += 64) {
        const int64_t c = c0 + lane;
        const uint64_t v = c < P.nchunks ? P.sums[c * nseq + u] : 0;
        uint64_t x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = shfl_up64(x, d);
            if (lane >= d) x = add_mod(x, y, G.p);
        }
        if (c < P.nchunks) P.sums[c * nseq + u] = add_mod(carry, sub_mod_p(x, v, G.p), G.p);
        carry = add_mod(carry, shfl64(x, 63), G.p);
    }
}

__global__ __launch_bounds__(256) void p2_glue_out_kernel(P2Glue G) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    GlueUnit U;
    if (!glue_unit(G, u, U)) return;
    const P2GluePart &P = G.part[U.part];
    if (U.kind == 1 && U.r >= G.m - 1) return;  // b has M - 1 columns
    uint64_t acc = P.sums[U.chunk * 4 * G.m + U.s];
    const bool direct = U.kind == 0 && U.r == G.m - 1;  // a_j[M - 1] = A_j[M - 1]
    const int64_t col = U.kind == 0 ? U.r : G.m + U.r;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < P2_CHUNK; ++q) {
        if (U.t0 + q >= U.t1) break;
        const int64_t j = U.par + 2 * (U.t0 + q);
        const uint64_t term = glue_term(P, G.m, G.p, U.kind, j, U.r);
        acc = add_mod(acc, term, G.p);
        const uint64_t val = direct ? term : acc;
        if (col < G.width)
            G.out[(P.row0 + j * P.rstep) * G.width + col] = val;
        else
            bad |= val != 0;
    }
    if (bad) set_status(G.devstat, KS_DEVSTAT_CHECK);
}

// ---- host launchers -----------------------------------------------------------------------------

// ---- Section 2.5: points in an extension of R ------------------------------------------------

// c v mod p for a small integer c (|c| <= 2)
__device__ __forceinline__ uint64_t small_mul(int c, uint64_t v, uint64_t p) {
    const uint64_t a = c == 0 ? 0 : (c == 2 || c == -2) ? add_mod(v, v, p) : v;
    return c < 0 ? (a ? p - a : 0) : a;
}

// Position i m + r of polynomial q of input w: sum over the rows reaching it (rows overlap
// when m < L_x), row i - t at column r + t m weighted by coef[q][(i - t) mod period]
__global__ __launch_bounds__(256) void p2_ext_eval_kernel(P2ExtEval E) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= 2 * E.np * E.le) return;
    const int64_t wq = t / E.le, pos = t - wq * E.le;
    const int w = (int)(wq / E.np), q = (int)(wq - (int64_t)w * E.np);
    const uint64_t *src = w ? E.g : E.f;
    const int64_t i = pos / E.m, r = pos - i * E.m;
    uint64_t acc = 0;
    bool bad = false;
    for (int64_t s = 0; i - s >= 0 && r + s * E.m < E.lx; ++s) {
        const int64_t row = i - s;
        if (row >= E.ly) continue;
        const uint64_t v = src[row * E.lx + r + s * E.m];
        bad |= v >= E.p;
        acc = add_mod(acc, small_mul(E.coef[q][row % E.period], v, E.p), E.p);
    }
    if (bad) set_status(E.devstat, KS_DEVSTAT_RANGE);
    E.out[wq * E.le + pos] = acc;
}

// first component of (c0 + c1 w)(a + b w) for c0, c1 in {-1, 0, 1}: c0 a - c1 b
__device__ __forceinline__ uint64_t wmul_re(int c0, int c1, uint64_t a, uint64_t b, uint64_t p) {
    uint64_t r = c0 > 0 ? a : c0 < 0 ? (a ? p - a : 0) : 0;
    if (c1 > 0) r = sub_mod_p(r, b, p);
    else if (c1 < 0) r = add_mod(r, b, p);
    return r;
}

__global__ __launch_bounds__(256) void p2_ext_readoff_kernel(P2ExtReadoff R) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= R.rows * R.width) return;
    const int64_t j = t / R.width, c = t - j * R.width;
    const int64_t pos = j * R.m + c;
    const uint64_t p = R.p;
    auto P = [&](int q) -> uint64_t { return pos < R.lh ? R.prod[q * R.lh + pos] : 0; };
    uint64_t v;
    if (!R.cube) {
        // h at y = x^m, -x^m and i x^m = re + i im (re = ac - bd, im = (a+b)(c+d) - ac - bd);
        // A_r = (H1 + (-1)^r H2 + 2 Re(i^-r (re + i im))) / 4
        const uint64_t h1 = P(0), h2 = P(1), ac = P(2), bd = P(3), s = P(4);
        const uint64_t re = sub_mod_p(ac, bd, p), im = sub_mod_p(sub_mod_p(s, ac, p), bd, p);
        const int rr = (int)(j & 3);
        const uint64_t e = (rr & 1) ? sub_mod_p(h1, h2, p) : add_mod(h1, h2, p);
        const uint64_t x = (rr & 1) ? im : re;
        const uint64_t x2 = add_mod(x, x, p);
        v = rr < 2 ? add_mod(e, x2, p) : sub_mod_p(e, x2, p);
    } else {
        // V_k = h at z^k x^m, z = 1 + w: V0 = H+, V3 = H-, V2 = (ac - bd, s - ac - 2 bd) at w,
        // V5 the same at -w, V4 and V1 their conjugates (a, b) -> (a - b, -b);
        // A_r = sum_k first component of (-w)^(r k) V_k (times 6^-1 below)
        uint64_t va[6], vb[6];
        va[0] = P(0);
        vb[0] = 0;
        va[3] = P(1);
        vb[3] = 0;
        {
            const uint64_t ac = P(2), bd = P(3), s = P(4);
            va[2] = sub_mod_p(ac, bd, p);
            vb[2] = sub_mod_p(sub_mod_p(s, ac, p), add_mod(bd, bd, p), p);
        }
        {
            const uint64_t ac = P(5), bd = P(6), s = P(7);
            va[5] = sub_mod_p(ac, bd, p);
            vb[5] = sub_mod_p(sub_mod_p(s, ac, p), add_mod(bd, bd, p), p);
        }
        va[4] = sub_mod_p(va[2], vb[2], p);
        vb[4] = vb[2] ? p - vb[2] : 0;
        va[1] = sub_mod_p(va[5], vb[5], p);
        vb[1] = vb[5] ? p - vb[5] : 0;
        // (-w)^e for e = 0..5 as (c0, c1): 1, -w, -1 - w, -1, w, 1 + w
        const int c0[6] = {1, 0, -1, -1, 0, 1}, c1[6] = {0, -1, -1, 0, 1, 1};
        const int rr = (int)(j % 6);
        v = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int e = (rr * k) % 6;
            v = add_mod(v, wmul_re(c0[e], c1[e], va[k], vb[k], p), p);
        }
    }
    // times 4^-1 (or 6^-1): v < p < 2^62 and inv < p, the product reduced by the 128-bit quotient
    R.out[t] = (uint64_t)(((unsigned __int128)v * R.inv) % p);
}

hipError_t launch_p2_ext_eval(const P2ExtEval &E, hipStream_t s) {
    const int64_t n = 2 * E.np * E.le;
    if (n <= 0) return hipSuccess;
    ks_launch(p2_ext_eval_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, E);
    return hipGetLastError();
}

hipError_t launch_p2_ext_readoff(const P2ExtReadoff &R, hipStream_t s) {
    const int64_t n = R.rows * R.width;
    if (n <= 0) return hipSuccess;
    ks_launch(p2_ext_readoff_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R);
    return hipGetLastError();
}

hipError_t launch_p2_eval(const P2Eval &E, hipStream_t s) {
    const int64_t n = 2 * E.k * E.le;
    if (n <= 0) return hipSuccess;
    ks_launch(p2_eval_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, E);
    return hipGetLastError();
}

hipError_t launch_p2_readoff(const P2Readoff &R, hipStream_t s) {
    const int64_t n = R.rows * R.width;
    if (n <= 0) return hipSuccess;
    ks_launch(p2_readoff_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R);
    return hipGetLastError();
}

hipError_t launch_p2_glue(const P2Glue &G, hipStream_t s) {
    const int64_t nseq = 4 * G.m;
    const int64_t n = G.part[0].nchunks * nseq + (G.nparts > 1 ? G.part[1].nchunks * nseq : 0);
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256));
    ks_launch(p2_glue_sum_kernel, grid, dim3(256), 0, s, G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ks_launch(p2_glue_scan_kernel, dim3((unsigned)((G.nparts * nseq + 3) / 4)), dim3(256), 0, s, G);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ks_launch(p2_glue_out_kernel, grid, dim3(256), 0, s, G);
    return hipGetLastError();
}

}  // namespace ks
