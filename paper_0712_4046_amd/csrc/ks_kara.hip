// ks_kara.hip -- one level of Karatsuba on the polynomials of a batch of modular products.
// Large products in (Z/pZ)[x] spend their time in the integer products, whose cost grows with
// the square of the length; splitting f and g at h = ceil(L / 2) turns one product of length L
// into three of length h (3/4 of the multiplication work) at the price of coefficient-wise
// additions mod p, which have no carries between coefficients and stream through HBM once.
// The three products run as an ordinary batch plan between the two kernels below.
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

__device__ __forceinline__ uint64_t kara_add(uint64_t a, uint64_t b, uint64_t p) {
    const uint64_t s = a + b;  // a, b < p < 2^62
    return s >= p ? s - p : s;
}
__device__ __forceinline__ uint64_t kara_sub(uint64_t a, uint64_t b, uint64_t p) { return a >= b ? a - b : a + p - b; }

// product blockIdx.y, term i: the halves and their sums (inputs are read once; a residue out
// of range is staged as it is and reported by the packing of the sub-products)
__global__ __launch_bounds__(256) void kara_split_kernel(const KaraProd *tab, const uint32_t *in, uint64_t *sub) {
    const KaraProd K = tab[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= K.h) return;
    const uint64_t *f = reinterpret_cast<const uint64_t *>(in + K.f_off);
    const uint64_t *g = reinterpret_cast<const uint64_t *>(in + K.g_off);
    const bool hi = K.h + i < K.L;
    const uint64_t f0 = f[i], f1 = hi ? f[K.h + i] : 0u;
    const uint64_t g0 = g[i], g1 = hi ? g[K.h + i] : 0u;
    uint64_t *o = sub + K.sub_in;
    o[i] = f0;
    o[K.h + i] = f1;
    o[2 * K.h + i] = kara_add(f0, f1, K.p);
    o[3 * K.h + i] = g0;
    o[4 * K.h + i] = g1;
    o[5 * K.h + i] = kara_add(g0, g1, K.p);
}

// coefficient k of f g from the three sub-products (each 2h - 1 residues)
__global__ __launch_bounds__(256) void kara_combine_kernel(const KaraProd *tab, const uint64_t *sub, uint32_t *out) {
    const KaraProd K = tab[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= 2 * K.L - 1) return;
    const int64_t m = 2 * K.h - 1;
    const uint64_t *z0 = sub + K.sub_out, *z2 = z0 + m, *z1 = z2 + m;
    uint64_t v = k < m ? z0[k] : 0u;
    const int64_t j = k - K.h;
    if (j >= 0 && j < m) v = kara_add(v, kara_sub(kara_sub(z1[j], z0[j], K.p), z2[j], K.p), K.p);
    const int64_t j2 = k - 2 * K.h;
    if (j2 >= 0 && j2 < m) v = kara_add(v, z2[j2], K.p);
    reinterpret_cast<uint64_t *>(out + K.h_off)[k] = v;
}

hipError_t launch_kara_split(const KaraProd *tab, int64_t count, int64_t max_h, const uint32_t *in, uint64_t *sub,
                             hipStream_t s) {
    if (count <= 0 || max_h <= 0) return hipSuccess;
    if (count > 65535) return hipErrorInvalidValue;
    ks_launch(kara_split_kernel, dim3((unsigned)((max_h + 255) / 256), (unsigned)count), dim3(256), 0, s, tab, in,
              sub);
    return hipGetLastError();
}

hipError_t launch_kara_combine(const KaraProd *tab, int64_t count, int64_t max_out, const uint64_t *sub,
                               uint32_t *out, hipStream_t s) {
    if (count <= 0 || max_out <= 0) return hipSuccess;
    if (count > 65535) return hipErrorInvalidValue;
    ks_launch(kara_combine_kernel, dim3((unsigned)((max_out + 255) / 256), (unsigned)count), dim3(256), 0, s, tab,
              sub, out);
    return hipGetLastError();
}

}  // namespace ks
