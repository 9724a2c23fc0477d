// valu_rates.hip -- issue rates of the vector-ALU instructions the kernels are built from, and
// of LDS reads in a few bank patterns, measured on the device (a measurement aid, built as libksprobe.so beside the library and
// driven by prof_tools.py; nothing in the library uses it).
//
// Each lane runs eight chains that feed each other (x[i] = op(x[i], x[i+1 mod 8])), so that no
// chain can be folded away by the compiler and eight independent instructions are ready at
// every step; a launch of `blocks` blocks of 256 threads runs `iters` steps of all eight.
// The rate of one operation is then blocks * 256 * iters * 8 / time lane-operations per second.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint32_t PRB_P = 998244353u;  // a prime below 2^30 (the transform engine's first)

__device__ __forceinline__ uint32_t pn_of(uint32_t p) {
    uint32_t x = p;
    for (int i = 0; i < 5; ++i) x *= 2u - p * x;
    return 0u - x;
}

template <int OP>
__global__ __launch_bounds__(256) void rate_kernel(uint64_t *out, uint32_t seed, int iters) {
    uint32_t a[8];
    uint64_t q[8];
    double d[8];
    for (int i = 0; i < 8; ++i) {
        a[i] = seed * 2654435761u + threadIdx.x * 8 + i;
        q[i] = ((uint64_t)a[i] << 17) ^ a[i];
        d[i] = 1.0 + 1e-9 * (double)a[i];
    }
    const uint32_t pn = pn_of(PRB_P);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = (i + 1) & 7;
            if (OP == 0) a[i] = a[i] + a[j];                                          // v_add_u32
            if (OP == 1) q[i] = q[i] + q[j];                                          // v_add_co + v_addc
            if (OP == 2) a[i] = min(a[i] - a[j], a[i]);                               // v_sub_u32 + v_min_u32
            if (OP == 3) a[i] = a[i] * a[j];                                          // v_mul_lo_u32
            if (OP == 4) a[i] = __umulhi(a[i], a[j]);                                 // v_mul_hi_u32
            if (OP == 5) q[i] = (uint64_t)(uint32_t)q[i] * (uint32_t)q[j] + q[i];     // v_mad_u64_u32
            if (OP == 6) d[i] = fma(d[i], d[j], -0.5);                                // v_fma_f64
            if (OP == 7) {                                                            // Montgomery product, no final subtraction
                const uint64_t t = (uint64_t)a[i] * (a[j] >> 2);
                const uint32_t m = (uint32_t)t * pn;
                a[i] = (uint32_t)((t + (uint64_t)m * PRB_P) >> 32);
            }
        }
    }
    uint64_t s = 0;
    for (int i = 0; i < 8; ++i) s += a[i] + q[i] + (uint64_t)d[i];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// LDS reads: every lane reads word addr(lane) + it 67 (mod 8192) of a 32 KiB buffer, the
// uniform shift keeping each step's bank pattern; the patterns tell how many banks serve a
// wave and how strided reads conflict.
template <int PAT>
__global__ __launch_bounds__(256) void lds_kernel(uint64_t *out, uint32_t seed, int iters) {
    __shared__ uint32_t buf[8192];
    for (int i = threadIdx.x; i < 8192; i += 256) buf[i] = i * seed;
    __syncthreads();
    const uint32_t l = threadIdx.x & 63;
    uint32_t a;
    if (PAT == 0) a = l;                               // consecutive words
    if (PAT == 1) a = 2 * l;                           // stride 2
    if (PAT == 2) a = 4 * l;                           // stride 4
    if (PAT == 3) a = 32 * l;                          // stride 32
    if (PAT == 4) a = (l & 31) + (l >> 5) * 128;       // two runs of 32 words, 128 apart
    if (PAT == 5) a = (l & 31) + (l >> 5) * 160;       // two runs of 32 words, 160 apart
    a += (threadIdx.x >> 6) * 1024;                    // each wave its own region
    uint32_t acc = 0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += buf[(a + (uint32_t)(it * 8 + u) * 67u) & 8191u];
    }
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

using KernelFn = void (*)(uint64_t *, uint32_t, int);
const KernelFn kKernels[] = {rate_kernel<0>, rate_kernel<1>, rate_kernel<2>, rate_kernel<3>, rate_kernel<4>,
                             rate_kernel<5>, rate_kernel<6>, rate_kernel<7>, lds_kernel<0>,  lds_kernel<1>,
                             lds_kernel<2>,  lds_kernel<3>,  lds_kernel<4>,  lds_kernel<5>};
const char *kNames[] = {"v_add_u32",
                        "v_add_co_u32 + v_addc_co_u32 (64-bit add)",
                        "v_sub_u32 + v_min_u32 (a partial reduction)",
                        "v_mul_lo_u32",
                        "v_mul_hi_u32",
                        "v_mad_u64_u32",
                        "v_fma_f64",
                        "Montgomery product without final subtraction (3 multiply-adds + 1 shift)",
                        "ds_read_b32, consecutive words",
                        "ds_read_b32, stride 2 words",
                        "ds_read_b32, stride 4 words",
                        "ds_read_b32, stride 32 words",
                        "ds_read_b32, two runs of 32 words 128 apart",
                        "ds_read_b32, two runs of 32 words 160 apart"};
// instructions per chain step (per LDS read for the LDS patterns)
const int kInsts[] = {1, 2, 2, 1, 1, 1, 1, 4, 1, 1, 1, 1, 1, 1};
constexpr int kCount = sizeof(kInsts) / sizeof(kInsts[0]);

}  // namespace

extern "C" {

int ks_probe_count(void) { return kCount; }
const char *ks_probe_name(int op) { return op >= 0 && op < kCount ? kNames[op] : ""; }
int ks_probe_insts(int op) { return op >= 0 && op < kCount ? kInsts[op] : 0; }

// Times `reps` launches of operation `op` (blocks of 256 threads, `iters` steps each) after one
// warm-up launch; *ms receives the average per launch.  Returns 0, or -1 on a bad argument or a
// HIP error.  Allocates and frees its own output buffer.
int ks_probe_valu(int op, int blocks, int iters, int reps, float *ms) {
    if (op < 0 || op >= kCount || blocks < 1 || iters < 1 || reps < 1 || !ms) return -1;
    uint64_t *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(uint64_t)) != hipSuccess) return -1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = -1;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        hipLaunchKernelGGL(kKernels[op], dim3(blocks), dim3(256), 0, 0, out, 3u, iters);
        bool ok = hipEventRecord(e0, 0) == hipSuccess;
        for (int r = 0; r < reps && ok; ++r) {
            hipLaunchKernelGGL(kKernels[op], dim3(blocks), dim3(256), 0, 0, out, 3u, iters);
            ok = hipGetLastError() == hipSuccess;
        }
        float t = 0.f;
        if (ok && hipEventRecord(e1, 0) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&t, e0, e1) == hipSuccess) {
            *ms = t / (float)reps;
            rc = 0;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}

}  // extern "C"
