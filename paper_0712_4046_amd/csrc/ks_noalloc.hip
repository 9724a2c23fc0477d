// ks_noalloc.hip -- ks_mul for callers that cannot allocate device memory.
//
// Everything a product needs beyond its inputs and output lives in one file-scope device array,
// `scratch`, of KS_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends):
//   [0, 256)                      control words: the device status word at 64, the ticket
//                                 counters of the pack and recombination blocks from 128
//   [256, 256 + 8 NA_STATUS)      look-back status words of the carry scans
//   [NA_WS, KS_NOALLOC_SCRATCH_BYTES)  the product's scratch regions (operands, column sums,
//                                 digits, recombined values, anchors, reconstruction buffers)
// The array's name is only a host-side stand-in, so its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and that address is what the jobs get.
// At that first use the control and status words are cleared by a fill kernel; later calls keep
// them valid without clearing: the ticket counters return to zero at the end of every launch,
// the look-back status words carry an epoch that grows by two per call, and the status word is
// cleared when it is read.  Every call on one GPU shares the array, so calls that may overlap on
// one GPU (other streams, other host threads) race; the caller orders them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/ks.h"
#include "ks_launch.h"
#include "ks_plan.h"

namespace ks {

constexpr int64_t NA_CTL = 256;           // control words
constexpr int64_t NA_STATUS = 1 << 16;    // look-back status words
constexpr int64_t NA_WS = NA_CTL + 8 * NA_STATUS;
static_assert(NA_WS % 256 == 0, "the product scratch must start 256-byte aligned");

static __device__ __align__(256) char scratch[KS_NOALLOC_SCRATCH_BYTES];

struct NoAllocDev {
    char *ptr = nullptr;  // the device address of `scratch` on this device
    Ctl ctl;
};
static std::mutex g_na_mu;
static NoAllocDev g_na[64];

// the device's copy of the array, set up on first use (with the device current)
static int noalloc_device(hipStream_t s, NoAllocDev **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KS_EHIP;
    NoAllocDev &D = g_na[dev];
    if (!D.ptr) {
        char *p = nullptr;
        if (hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return KS_EHIP;
        // control and status words start at zero (epoch 0 is never a fresh status word)
        if (launch_fill_zero(reinterpret_cast<uint64_t *>(p), NA_WS / 8, s) != hipSuccess) return KS_EHIP;
        D.ctl.devstat = reinterpret_cast<uint32_t *>(p + 64);
        D.ctl.ctrs = reinterpret_cast<uint64_t *>(p + 128);
        D.ctl.status = reinterpret_cast<uint64_t *>(p + NA_CTL);
        D.ctl.status_words = NA_STATUS;
        D.ctl.epoch = 0;
        D.ptr = p;
    }
    *out = &D;
    return KS_OK;
}

// status word of the array on the current device, read and cleared after syncing `s` (KS_OK
// when this device never ran ks_mul_noalloc)
int noalloc_status(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KS_EHIP;
    uint32_t *w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_na_mu);
        if (!g_na[dev].ptr) return KS_OK;
        w = g_na[dev].ctl.devstat;
    }
    return read_status(w, s);
}

}  // namespace ks

using namespace ks;

extern "C" int ks_mul_noalloc(const uint32_t *f, const uint32_t *g, int64_t len_f, int64_t len_g, int32_t coeff_bits,
                              int32_t variant, void *stream, uint32_t *h) {
    if (!f || !g || !h) return KS_EINVAL;
    int rc = validate_spec(len_f, len_g, coeff_bits, variant, true);
    if (rc != KS_OK) return rc;
    if (device_ok() != 1) return KS_EUNSUPPORTED;
    Spec sp{len_f, len_g, coeff_bits, (int)((coeff_bits + 31) / 32), (variant & KS_SIGNED) != 0, 0,
            variant & KS_VARIANT_MASK, variant & KS_ENGINE_ANY};
    Geom G;
    rc = plan_product(sp, G);
    if (rc != KS_OK) return rc;
    // the product's scratch regions end where its status words would start; those have their
    // own part of the array
    if (G.ws_status > KS_NOALLOC_SCRATCH_BYTES - NA_WS ||
        std::max<int64_t>(std::max(G.pack_blocks, G.norm_blocks + G.norm_status_extra), 1) > NA_STATUS)
        return KS_ESCRATCH;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_na_mu);
    NoAllocDev *D = nullptr;
    rc = noalloc_device(s, &D);
    if (rc != KS_OK) return rc;
    return run_product(G, f, g, h, D->ptr + NA_WS, D->ctl, s);
}
